// Tail-colour network f(x) of STAR-NT (Sec. 3.3) at full resolution, over the
// bilinearly upscaled pass-3 features (Sec. 3.2). Three dense layers with ReLU
// after each; x = (N, t_tail, Ct_rgb) plus zero padding to 16 inputs.
// Optionally fused with the eq (3) composite (starnt_infer_composite), which
// saves writing and re-reading the tail colour and the second feature fetch.
//
// Paths:
//  * STARNT_F32  : one thread per pixel, FP32 FMAs, weights read with
//                  wave-uniform addresses (scalar loads).
//  * STARNT_BF16 : matrix cores. Pixels are the N dimension of
//                  v_mfma_f32_32x32x16_bf16 (32 pixels per wave step); a layer
//                  is H^T = W H_prev^T. The hidden units of layer 1 are stored
//                  in a permuted order chosen so that each lane's accumulator
//                  registers of layer 1 are exactly its B-operand registers of
//                  layer 2 (and layer 2's of layer 3): no data moves between
//                  lanes. The 3-wide output layer is a 32-row tile with
//                  rows 0..2 live.
//  * STARNT_FP8  : the same structure with OCP E4M3 operands and per-layer
//                  scales on v_mfma_f32_32x32x16_fp8_fp8.
// Weights are staged once per block in LDS; blocks are persistent and walk
// 64-pixel steps.
#include <type_traits>

#include "internal.h"

namespace starnt {
namespace {

// what a kernel produces: the tail colour (starnt_infer), the eq (3)
// composite with it, or the DFAOIT composite (eq (2))
constexpr int kTail = 0, kComp = 1, kDfa = 2, kSel = 3;  // kSel: kComp, network only off flat cells
constexpr int kPatch = 4;  // kComp over a pixel list: compact full-resolution inputs

struct InferArgs {
  int W, H;
  const float4* tail;
  const float4* tail_avg;  // tail means (DFAOIT only)
  const uint8_t* level;    // leaf level per quadtree cell (selective only)
  int cs, Cw;              // cell side in pixels, cells per row
  const uint32_t* count;
  const float4* layer1;
  const float4* layer2;
  const starnt_sched* sched;
  const float* __restrict__ W1;
  const float* __restrict__ b1;
  const float* __restrict__ W2;
  const float* __restrict__ b2;
  const float* __restrict__ W3;
  const float* __restrict__ b3;
  int in, h1, h2;
  float sa[3], sw[3];  // FP8 scales
  float bg0, bg1, bg2;
  float* out;          // tail colour [P][3] or composite rgb [P][3]
  const uint32_t* list;    // kPatch: slot i holds pixel list[i] of the frame
  const uint32_t* list_n;  // kPatch: number of slots in use (device)
  uint32_t frame_p;        // kPatch: pixels of the output frame
};

// pixels a launch covers: the frame, or the slots of the list in use
template <int MODE>
__device__ __forceinline__ int pixel_count(const InferArgs& a) {
  if constexpr (MODE == kPatch) {
    const uint32_t n = *a.list_n, cap = (uint32_t)a.W;
    return (int)(n < cap ? n : cap);
  }
  return a.W * a.H;
}

// inputs of one pixel for the network and the composite
struct PixIn {
  uint32_t n;
  float x[11];         // upscaled network input (n >= 3): 5 values, or 11 (DFAOIT)
  float tt;            // upscaled t_tail (n >= 3)
  float4 l1;           // layer 1 (composite only)
  float4 l2;           // upscaled layer 2 (composite only)
  float e0, e1, e2;    // exact two-layer colour (DFAOIT only)
  bool flat;           // in a level-0 quadtree leaf (selective only)
};

__device__ __forceinline__ float lerp1(float p, float q, float w) { return fmaf(w, q - p, p); }
__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float w) {
  return make_float4(lerp1(a.x, b.x, w), lerp1(a.y, b.y, w), lerp1(a.z, b.z, w), lerp1(a.w, b.w, w));
}

// Raw inputs of one pixel: all loads are issued up front, independent of the
// loaded values, so a prefetched group costs one memory round trip.
struct PixRaw {
  uint32_t n;
  float4 t[4];   // (N, t_tail, Ct_r, Ct_g) of the four pass-3 taps
  float2 t4[4];  // (Ct_b, A) of the four taps (A: DFAOIT only)
  float4 av[4];  // tail means of the four taps (DFAOIT only)
  float4 l1;
  float4 l2[4];  // the four pass-2 taps
  float wx3, wy3, wx2, wy2;
  uint32_t lvl;  // leaf level of the pixel's quadtree cell (selective only)
};

// Which grids are at full resolution (wave-uniform, fixed for a launch): a
// full-resolution grid's sample for pixel p is p itself, so its taps are not
// computed, only one is loaded, and the blend takes it as it is (the same
// value the bilinear blend gives with weight 0).
struct Full {
  bool g2, g3;
};
template <int MODE>
__device__ __forceinline__ Full full_grids(const InferArgs& a, const Grids& g) {
  if constexpr (MODE == kPatch) return Full{true, true};
  return Full{g.w2 == a.W && g.h2 == a.H, g.w3 == a.W && g.h3 == a.H};
}
// The same choice fixed at compile time, for loops specialised per case: with
// no merge of the two load paths inside the loop, a prefetched step's loads
// stay in flight in their own registers until the step is used.
template <bool G2, bool G3>
struct FullC {
  static constexpr bool g2 = G2, g3 = G3;
};

template <int MODE, class F>
__device__ __forceinline__ void issue_loads(const InferArgs& a, const Grids& g, const F& f, int p, PixRaw& r) {
  r.n = a.count[p];
  if constexpr (MODE == kPatch) {
    // slot p holds its own full-resolution features
    r.t[0] = a.tail[2u * p];
    r.t4[0] = make_float2(a.tail[2u * p + 1u].x, 0.0f);
    r.l2[0] = a.layer2[p];
    r.l1 = a.layer1[p];
    return;
  }
  int x, y;
  pixel_xy(p, a.W, x, y);
  if (f.g3) {
    r.t[0] = a.tail[2u * p];
    const float4 hi = a.tail[2u * p + 1u];
    r.t4[0] = make_float2(hi.x, MODE == kDfa ? hi.y : 0.0f);
    if constexpr (MODE == kDfa) r.av[0] = a.tail_avg[p];
  } else {
    const Taps tx = axis_taps(x, a.W, g.w3), ty = axis_taps(y, a.H, g.h3);
    // grid sides are at most 16384, so sample indices fit 32 bits
    const uint32_t r0 = mul24((uint32_t)ty.i0, (uint32_t)g.w3), r1 = mul24((uint32_t)ty.i1, (uint32_t)g.w3);
    const uint32_t i3[4] = {r0 + tx.i0, r0 + tx.i1, r1 + tx.i0, r1 + tx.i1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = i3[k];
      r.t[k] = a.tail[2u * i];
      const float4 hi = a.tail[2u * i + 1u];
      r.t4[k] = make_float2(hi.x, MODE == kDfa ? hi.y : 0.0f);
      if constexpr (MODE == kDfa) r.av[k] = a.tail_avg[i];
    }
    r.wx3 = tx.w1;
    r.wy3 = ty.w1;
  }
  if constexpr (MODE == kSel) r.lvl = a.level[(y / a.cs) * a.Cw + x / a.cs];
  if constexpr (MODE >= kComp) {
    r.l1 = a.layer1[p];
    if (f.g2) {
      r.l2[0] = a.layer2[p];
    } else {
      const Taps ux = axis_taps(x, a.W, g.w2), uy = axis_taps(y, a.H, g.h2);
      const uint32_t r0 = mul24((uint32_t)uy.i0, (uint32_t)g.w2), r1 = mul24((uint32_t)uy.i1, (uint32_t)g.w2);
      const uint32_t i2[4] = {r0 + ux.i0, r0 + ux.i1, r1 + ux.i0, r1 + ux.i1};
#pragma unroll
      for (int k = 0; k < 4; ++k) r.l2[k] = a.layer2[i2[k]];
      r.wx2 = ux.w1;
      r.wy2 = uy.w1;
    }
  }
}

// bilinear blend of the raw taps; the full-resolution count gates the terms
__device__ __forceinline__ float blend4(float p0, float p1, float p2, float p3, float wx, float wy) {
  return lerp1(lerp1(p0, p1, wx), lerp1(p2, p3, wx), wy);
}

template <int MODE, class F>
__device__ __forceinline__ PixIn blend(const PixRaw& r, const F& f) {
  PixIn in;
  in.n = r.n;
  in.flat = MODE == kSel && r.lvl == 0;
#pragma unroll
  for (int e = 0; e < 11; ++e) in.x[e] = 0.0f;
  in.tt = 1.0f;
  if (r.n >= 3) {
    float4 v;
    float cb;
    if (f.g3) {
      v = r.t[0];
      cb = r.t4[0].x;
    } else {
      v = lerp4(lerp4(r.t[0], r.t[1], r.wx3), lerp4(r.t[2], r.t[3], r.wx3), r.wy3);
      cb = blend4(r.t4[0].x, r.t4[1].x, r.t4[2].x, r.t4[3].x, r.wx3, r.wy3);
    }
    in.tt = v.y;
    if constexpr (MODE == kDfa) {
      // x = (exact two-layer colour, tail mean colour, tail mean opacity,
      // tail accumulated colour S = Ct A, N); S is formed per tap and then
      // blended like every other input
      float4 av;
      float s0, s1, s2;
      if (f.g3) {
        av = r.av[0];
        s0 = r.t[0].z * r.t4[0].y;
        s1 = r.t[0].w * r.t4[0].y;
        s2 = r.t4[0].x * r.t4[0].y;
      } else {
        av = lerp4(lerp4(r.av[0], r.av[1], r.wx3), lerp4(r.av[2], r.av[3], r.wx3), r.wy3);
        s0 = blend4(r.t[0].z * r.t4[0].y, r.t[1].z * r.t4[1].y, r.t[2].z * r.t4[2].y, r.t[3].z * r.t4[3].y,
                    r.wx3, r.wy3);
        s1 = blend4(r.t[0].w * r.t4[0].y, r.t[1].w * r.t4[1].y, r.t[2].w * r.t4[2].y, r.t[3].w * r.t4[3].y,
                    r.wx3, r.wy3);
        s2 = blend4(r.t4[0].x * r.t4[0].y, r.t4[1].x * r.t4[1].y, r.t4[2].x * r.t4[2].y, r.t4[3].x * r.t4[3].y,
                    r.wx3, r.wy3);
      }
      in.x[3] = av.x; in.x[4] = av.y; in.x[5] = av.z; in.x[6] = av.w;
      in.x[7] = s0;
      in.x[8] = s1;
      in.x[9] = s2;
      in.x[10] = v.x;
    } else {
      in.x[0] = v.x; in.x[1] = v.y; in.x[2] = v.z; in.x[3] = v.w;
      in.x[4] = cb;
    }
  }
  if constexpr (MODE >= kComp) {
    in.l1 = r.l1;
    in.l2 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r.n >= 2)
      in.l2 = f.g2 ? r.l2[0] : lerp4(lerp4(r.l2[0], r.l2[1], r.wx2), lerp4(r.l2[2], r.l2[3], r.wx2), r.wy2);
  }
  if constexpr (MODE == kDfa) {
    const float om1 = 1.0f - in.l1.w;
    in.e0 = fmaf(om1, in.l2.x, in.l1.x);
    in.e1 = fmaf(om1, in.l2.y, in.l1.y);
    in.e2 = fmaf(om1, in.l2.z, in.l1.z);
    if (r.n >= 3) { in.x[0] = in.e0; in.x[1] = in.e1; in.x[2] = in.e2; }
  }
  return in;
}

template <int MODE>
__device__ __forceinline__ void load_pixel(const InferArgs& a, const Grids& g, int p, PixIn& in) {
  PixRaw r;
  const Full f = full_grids<MODE>(a, g);
  issue_loads<MODE>(a, g, f, p, r);
  in = blend<MODE>(r, f);
}

// write the tail colour, the eq (3) composite with it, or the DFAOIT
// composite (eq (2)): C_t + C_b prod(1 - a), with C_t the network's colour
// where N >= 3 and the exact two-layer colour elsewhere
template <int MODE>
__device__ __forceinline__ void store_pixel(const InferArgs& a, int p, const PixIn& in, float f0, float f1, float f2) {
  const bool on = in.n >= 3;
  size_t dst = (size_t)p;
  if constexpr (MODE == kPatch) {
    dst = a.list[p];
    if (dst >= a.frame_p) return;  // flagged by the list's feature pass
  }
  float* o = a.out + 3 * dst;
  if constexpr (MODE == kDfa) {
    const float T = (1.0f - in.l1.w) * (1.0f - in.l2.w) * (on ? in.tt : 1.0f);
    o[0] = fmaf(T, a.bg0, on ? f0 : in.e0);
    o[1] = fmaf(T, a.bg1, on ? f1 : in.e1);
    o[2] = fmaf(T, a.bg2, on ? f2 : in.e2);
  } else {
    if (!on) { f0 = f1 = f2 = 0.0f; }
    if constexpr (MODE == kSel) {
      // flat cells take the order-free tail estimate f_avg = Ct (1 - t_tail)
      if (in.flat) {
        const float w = 1.0f - in.tt;
        f0 = on ? in.x[2] * w : 0.0f;
        f1 = on ? in.x[3] * w : 0.0f;
        f2 = on ? in.x[4] * w : 0.0f;
      }
    }
    if constexpr (MODE == kComp || MODE == kSel || MODE == kPatch) {
      const float tt = on ? in.tt : 1.0f;
      const float om1 = 1.0f - in.l1.w;
      const float T2 = om1 * (1.0f - in.l2.w);
      const float Tb = T2 * tt;
      o[0] = in.l1.x + om1 * in.l2.x + T2 * f0 + Tb * a.bg0;
      o[1] = in.l1.y + om1 * in.l2.y + T2 * f1 + Tb * a.bg1;
      o[2] = in.l1.z + om1 * in.l2.z + T2 * f2 + Tb * a.bg2;
    } else {
      o[0] = f0;
      o[1] = f1;
      o[2] = f2;
    }
  }
}

// output activation: ReLU (STAR-NT) or the logistic sigmoid (DFAOIT)
template <int MODE>
__device__ __forceinline__ float out_act(float z) {
  if constexpr (MODE == kDfa) return 1.0f / (1.0f + __expf(-z));
  else return fmaxf(z, 0.0f);
}

// number of network inputs in use
template <int MODE>
constexpr int n_inputs() { return MODE == kDfa ? 11 : 5; }

// ---------------------------------------------------------------------------
// FP32 VALU path

template <int H1, int H2, int MODE>
__global__ __launch_bounds__(256) void infer_f32_kernel(InferArgs a) {
  const int P = pixel_count<MODE>(a);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const Grids g = load_grids(a.sched, a.W, a.H);
  PixIn in;
  load_pixel<MODE>(a, g, p, in);
  float o0 = 0.f, o1 = 0.f, o2 = 0.f;
  if (in.n >= 3 && !in.flat) {
    float h1[H1];
#pragma unroll
    for (int j = 0; j < H1; ++j) {
      float s = a.b1[j];
#pragma unroll
      for (int i = 0; i < n_inputs<MODE>(); ++i) s = fmaf(a.W1[j * a.in + i], in.x[i], s);
      h1[j] = fmaxf(s, 0.0f);
    }
    float h2[H2];
#pragma unroll
    for (int k = 0; k < H2; ++k) {
      float s = a.b2[k];
#pragma unroll
      for (int j = 0; j < H1; ++j) s = fmaf(a.W2[k * H1 + j], h1[j], s);
      h2[k] = fmaxf(s, 0.0f);
    }
    float s0 = a.b3[0], s1 = a.b3[1], s2 = a.b3[2];
#pragma unroll
    for (int k = 0; k < H2; ++k) {
      s0 = fmaf(a.W3[k], h2[k], s0);
      s1 = fmaf(a.W3[H2 + k], h2[k], s1);
      s2 = fmaf(a.W3[2 * H2 + k], h2[k], s2);
    }
    o0 = out_act<MODE>(s0);
    o1 = out_act<MODE>(s1);
    o2 = out_act<MODE>(s2);
  }
  store_pixel<MODE>(a, p, in, o0, o1, o2);
}

// ---------------------------------------------------------------------------
// matrix-core paths (BF16 and FP8)

// b = p[0] + p[1] + p[2] exactly, each part a bf16 value: p[0] is b rounded
// to bf16 (8 significant bits), p[1] the remainder (at most 16 significant
// bits, exact in FP32) rounded likewise, p[2] what is left (at most 8 bits)
__device__ __forceinline__ void bias_parts(float b, float* p) {
  p[0] = (float)static_cast<__bf16>(b);
  const float r = b - p[0];
  p[1] = (float)static_cast<__bf16>(r);
  p[2] = r - p[1];
}

template <bool FP8>
struct Op {
  using vec = typename std::conditional<FP8, fp8x8, bf16x8>::type;
};

template <bool FP8>
__device__ __forceinline__ void set8(typename Op<FP8>::vec& v, const float* w, float scale_inv) {
  if constexpr (FP8) {
    const uint32_t lo = e4m3_pack4(sat448(w[0] * scale_inv), sat448(w[1] * scale_inv), sat448(w[2] * scale_inv),
                                   sat448(w[3] * scale_inv));
    const uint32_t hi = e4m3_pack4(sat448(w[4] * scale_inv), sat448(w[5] * scale_inv), sat448(w[6] * scale_inv),
                                   sat448(w[7] * scale_inv));
    v = (long)(((unsigned long)hi << 32) | lo);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = static_cast<__bf16>(w[e]);
  }
}

// ReLU then pack: FP8 clamps in FP32 before the convert; BF16 converts first
// and zeroes negative values on the packed bits (a bf16 value is negative,
// -0 included, exactly when its 16-bit pattern is a negative integer), two
// values per instruction
template <bool FP8>
__device__ __forceinline__ void set8_relu(typename Op<FP8>::vec& v, float* w, float scale_inv) {
  if constexpr (FP8) {
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = fmaxf(w[e], 0.0f);
    set8<FP8>(v, w, scale_inv);
  } else {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    i32x4 packed;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bf16x2 b = __builtin_convertvector((f32x2){w[2 * e], w[2 * e + 1]}, bf16x2);
      const s16x2 r = __builtin_elementwise_max(__builtin_bit_cast(s16x2, b), (s16x2)0);
      packed[e] = __builtin_bit_cast(int, r);
    }
    v = __builtin_bit_cast(bf16x8, packed);
  }
}

template <bool FP8>
__device__ __forceinline__ f32x16 mfma(const typename Op<FP8>::vec& A, const typename Op<FP8>::vec& B, f32x16 c) {
  if constexpr (FP8) return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(A, B, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, c, 0, 0, 0);
}

constexpr int kMaxParams = 64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3;

// T1, T2: number of 32-row tiles of the two hidden layers (h padded with zero
// weights up to 32 * T). All three layers run on the matrix cores; the rows of
// both hidden layers are stored permuted (perm_row) so each layer's
// accumulators are the next layer's B operand in place. The 3-wide output
// layer is a 32-row tile with rows 0..2 live: lane half 0 holds a pixel's
// three outputs in accumulator registers 0..2.
// A wave step covers 64 pixels: every lane loads its own pixel, the second
// 32-pixel group's inputs cross to lane half 0 with one xor-32 shuffle, and
// its outputs cross back the same way.
// The 32-wide networks are held to 3 waves per SIMD (at most 168 VGPRs; a few
// variants spill a few dwords for it); at 4 waves (128 VGPRs) the BF16
// composite measured slower.
template <int T1, int T2, bool FP8, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(T1 * T2 == 1 ? 3 : 1)))
void infer_mfma_kernel(InferArgs a) {
  __shared__ float s_w[kMaxParams];
  using V = typename Op<FP8>::vec;
  // stage weights: W1 [h1][16], b1, W2 [h2][h1], b2, W3 [3][h2], b3
  const int nW1 = a.h1 * 16, nW2 = a.h2 * a.h1, nW3 = 3 * a.h2;
  float* sW1 = s_w;
  float* sb1 = sW1 + nW1;
  float* sW2 = sb1 + a.h1;
  float* sb2 = sW2 + nW2;
  float* sW3 = sb2 + a.h2;
  float* sb3 = sW3 + nW3;
  for (int i = threadIdx.x; i < nW1; i += blockDim.x) sW1[i] = a.W1[i];
  for (int i = threadIdx.x; i < a.h1; i += blockDim.x) sb1[i] = a.b1[i];
  for (int i = threadIdx.x; i < nW2; i += blockDim.x) sW2[i] = a.W2[i];
  for (int i = threadIdx.x; i < a.h2; i += blockDim.x) sb2[i] = a.b2[i];
  for (int i = threadIdx.x; i < nW3; i += blockDim.x) sW3[i] = a.W3[i];
  for (int i = threadIdx.x; i < 3; i += blockDim.x) sb3[i] = a.b3[i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int waves_per_block = blockDim.x >> 6;
  const int P = pixel_count<MODE>(a);
  const int nsteps = (P + 63) / 64;
  // Steps of 64 pixels: blocks go to the eight XCDs in turn, so with a grid
  // of a multiple of 8 blocks each XCD takes a contiguous eighth of the
  // steps (its waves stride through it). Vertically adjacent steps then
  // share the pass-3 rows their taps read in one XCD's L2 instead of
  // fetching them into several.
  int wave, nwaves, st_end;
  if ((gridDim.x & 7) == 0 && MODE != kPatch) {
    const int xcd = (int)(blockIdx.x & 7);
    const int lo = (int)(((long long)nsteps * xcd) >> 3);
    st_end = (int)(((long long)nsteps * (xcd + 1)) >> 3);
    wave = lo + (int)(blockIdx.x >> 3) * waves_per_block + (int)(threadIdx.x >> 6);
    nwaves = (int)(gridDim.x >> 3) * waves_per_block;
  } else {
    wave = blockIdx.x * waves_per_block + (threadIdx.x >> 6);
    nwaves = gridDim.x * waves_per_block;
    st_end = nsteps;
  }
  const Grids g = load_grids(a.sched, a.W, a.H);
  // FP8: activation scale of each layer's input, inverse weight scale, and
  // the dequantisation factor sa * sw of each layer's products
  const float ia0 = FP8 ? 1.0f / a.sa[0] : 1.0f, ia1 = FP8 ? 1.0f / a.sa[1] : 1.0f;
  const float ia2 = FP8 ? 1.0f / a.sa[2] : 1.0f;
  const float iw0 = FP8 ? 1.0f / a.sw[0] : 1.0f, iw1 = FP8 ? 1.0f / a.sw[1] : 1.0f;
  const float iw2 = FP8 ? 1.0f / a.sw[2] : 1.0f;
  const float dq0 = FP8 ? a.sa[0] * a.sw[0] : 1.0f, dq1 = FP8 ? a.sa[1] * a.sw[1] : 1.0f;
  const float dq2 = FP8 ? a.sa[2] * a.sw[2] : 1.0f;

  // ---- weights into registers, in operand layout ----
  // BF16: the hidden layers' FP32 biases enter the matrix-core accumulation
  // as three bf16 parts that sum to them exactly, one per K slot, against
  // inputs of 1 (layer 1: the free K slots after the inputs; layer 2: one
  // extra K chunk). FP8 adds them after the dequantisation.
  constexpr int NIN = n_inputs<MODE>();
  constexpr int NB = FP8 ? 0 : 3;
  // layer 1: tile t, physical row `col` = hidden unit 32 t + perm_row(col)
  V A1[T1];
  f32x16 B1v[T1];
#pragma unroll
  for (int t = 0; t < T1; ++t) {
    const int u = 32 * t + perm_row(col);
    float w[8];
    float bp[3] = {0.0f, 0.0f, 0.0f};
    if (NB && u < a.h1) bias_parts(sb1[u], bp);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * half + e;
      w[e] = (u < a.h1 && k < NIN) ? sW1[u * 16 + k] : (k >= NIN && k < NIN + NB ? bp[k - NIN < 3 ? k - NIN : 0] : 0.0f);
    }
    set8<FP8>(A1[t], w, iw0);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int uu = 32 * t + perm_row(8 * (v >> 2) + 4 * half + (v & 3));
      B1v[t][v] = uu < a.h1 ? sb1[uu] : 0.0f;
    }
  }
  // layer 2: tile t, physical row `col` = unit 32 t + perm_row(col); K chunk c
  // runs over layer-1 units 16 c + 8 half + e
  constexpr int C2 = 2 * T1;
  V A2[T2][C2];
  V A2b[T2];  // BF16: bias parts of unit u in K slots 0..2 of lane half 0
  f32x16 B2v[T2];
#pragma unroll
  for (int t = 0; t < T2; ++t) {
    const int u = 32 * t + perm_row(col);
    {
      float bp[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      if (NB && half == 0 && u < a.h2) bias_parts(sb2[u], bp);
      set8<FP8>(A2b[t], bp, 1.0f);
    }
#pragma unroll
    for (int c = 0; c < C2; ++c) {
      float w[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * c + 8 * half + e;
        w[e] = (u < a.h2 && k < a.h1) ? sW2[u * a.h1 + k] : 0.0f;
      }
      set8<FP8>(A2[t][c], w, iw1);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int uu = 32 * t + perm_row(8 * (v >> 2) + 4 * half + (v & 3));
      B2v[t][v] = uu < a.h2 ? sb2[uu] : 0.0f;
    }
  }
  // layer 3: rows 0..2 live, K chunk c over layer-2 units 16 c + 8 half + e
  constexpr int C3 = 2 * T2;
  V A3[C3];
#pragma unroll
  for (int c = 0; c < C3; ++c) {
    float w[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 16 * c + 8 * half + e;
      w[e] = (col < 3 && k < a.h2) ? sW3[col * a.h2 + k] : 0.0f;
    }
    set8<FP8>(A3[c], w, iw2);
  }
  const float b30 = sb3[0], b31 = sb3[1], b32 = sb3[2];
  V ONES;  // B operand of the layer-2 bias chunk
  {
    const float one[8] = {1.0f, 1.0f, 1.0f, 1.0f, 1.0f, 1.0f, 1.0f, 1.0f};
    set8<FP8>(ONES, one, 1.0f);
  }

  // the network on one 32-pixel group; xv holds this lane's half of the
  // group's K inputs (half 0: inputs 0..7, half 1: inputs 8..15)
  auto net = [&](const float xv[8], float& o0, float& o1, float& o2) {
    V X;
    {
      float xx[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xx[e] = xv[e];
      set8<FP8>(X, xx, ia0);
    }
    V Hb[C2];
#pragma unroll
    for (int t = 0; t < T1; ++t) {
      f32x16 acc = {};
      acc = mfma<FP8>(A1[t], X, acc);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[e] = NB ? acc[8 * c + e] : fmaf(acc[8 * c + e], dq0, B1v[t][8 * c + e]);
        set8_relu<FP8>(Hb[2 * t + c], hv, ia1);
      }
    }
    V Hb2[C3];
#pragma unroll
    for (int t = 0; t < T2; ++t) {
      f32x16 acc = {};
      if constexpr (NB != 0) acc = mfma<FP8>(A2b[t], ONES, acc);
#pragma unroll
      for (int c = 0; c < C2; ++c) acc = mfma<FP8>(A2[t][c], Hb[c], acc);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) hv[e] = NB ? acc[8 * c + e] : fmaf(acc[8 * c + e], dq1, B2v[t][8 * c + e]);
        set8_relu<FP8>(Hb2[2 * t + c], hv, ia2);
      }
    }
    f32x16 acc = {};
#pragma unroll
    for (int c = 0; c < C3; ++c) acc = mfma<FP8>(A3[c], Hb2[c], acc);
    o0 = out_act<MODE>(fmaf(acc[0], dq2, b30));
    o1 = out_act<MODE>(fmaf(acc[1], dq2, b31));
    o2 = out_act<MODE>(fmaf(acc[2], dq2, b32));
  };

  // software pipeline: the loads of the wave's next step are in flight while
  // the network runs on the current one
  // The loads are unconditional (a branch around them would merge register
  // sets and wait on the loads there): a lane past the end loads pixel P - 1,
  // and the wave's last step prefetches its own pixels again (cache hits);
  // neither is used.
  auto run = [&](auto full) {
  if (wave >= st_end) return;
  PixRaw r;
  int pn = wave * 64 + lane;
  issue_loads<MODE>(a, g, full, pn < P ? pn : P - 1, r);
  for (int st = wave; st < st_end; st += nwaves) {
    const int p = pn;
    const bool live = p < P;
    const PixIn in = blend<MODE>(r, full);
    const int sn = st + nwaves;
    pn = sn * 64 + lane;
    const int q = sn < st_end ? pn : p;
    issue_loads<MODE>(a, g, full, q < P ? q : P - 1, r);
    // group A is the pixels of lanes 0..31, group B those of lanes 32..63; a
    // group's inputs 0..7 go to half 0 and 8..15 to half 1 of the same
    // column, so each lane exchanges one half with its xor-32 partner
    const bool need = live && in.n >= 3 && !in.flat;
    // K slots past the inputs: 1 in the layer-1 bias slots, else 0
    auto cst = [](int k) { return k >= NIN && k < NIN + NB ? 1.0f : 0.0f; };
    float own[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) own[e] = e < NIN ? (need ? in.x[e < 11 ? e : 0] : 0.0f) : cst(e);
    float xa[8], xb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float lo = own[e], hi = own[8 + e];
      const float lo_x = e < NIN ? __shfl_xor(lo, 32) : cst(e);
      const float hi_x = 8 + e < NIN ? __shfl_xor(hi, 32) : cst(8 + e);
      xa[e] = half == 0 ? lo : hi_x;
      xb[e] = half == 0 ? lo_x : hi;
    }
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f;
    // (selective: a step with no pixel off the flat cells skips the network)
    if (MODE != kSel || __builtin_amdgcn_ballot_w64(need) != 0) {
      net(xa, a0, a1, a2);   // group A, outputs in half 0
      net(xb, b0, b1, b2);   // group B, outputs in half 0
    }
    b0 = __shfl_xor(b0, 32);
    b1 = __shfl_xor(b1, 32);
    b2 = __shfl_xor(b2, 32);
    if (live) {
      if (half == 0) store_pixel<MODE>(a, p, in, a0, a1, a2);
      else store_pixel<MODE>(a, p, in, b0, b1, b2);
    }
  }
  };
  // one loop per case (wave-uniform). A full-resolution pass-3 grid under a
  // reduced pass-2 grid takes the general loop: its taps are the sample
  // itself and its second tap has weight 0, which the blend returns exactly.
  const Full full = full_grids<MODE>(a, g);
  if (full.g2 && full.g3) run(FullC<true, true>{});
  else if (full.g2) run(FullC<true, false>{});
  else run(FullC<false, false>{});
}

template <int H1, int H2, int MODE>
void launch_f32(const InferArgs& a, hipStream_t s) {
  const int P = a.W * a.H;
  launch_maybe_timed(take_launch_timer(), infer_f32_kernel<H1, H2, MODE>, dim3((P + 255) / 256), dim3(256), s, a);
}

// blocks of 256 threads of `kernel` that the device holds at once (the
// occupancy the register count allows, times the CUs), cached per device
template <typename K>
int resident_blocks(K kernel) {
  static int cache[16] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) dev = 0;
  if (cache[dev] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    cache[dev] = per_cu * cus;
  }
  return cache[dev];
}

template <int T1, int T2, bool FP8, int MODE>
void launch_mfma(const InferArgs& a, hipStream_t s) {
  const int P = a.W * a.H;
  const int steps = (P + 63) / 64;
  // persistent blocks, exactly as many as are resident at once: a second
  // partial round of blocks would run nearly alone at the end
  int blocks = (steps + 3) / 4;
  const int resident = resident_blocks(infer_mfma_kernel<T1, T2, FP8, MODE>);
  if (blocks > resident) blocks = resident;
  // a pixel list is usually a small part of the frame: fewer blocks, so each
  // wave's weight set-up serves several steps (measured best at 1080p with
  // 5-10% of the pixels listed)
  if (MODE == kPatch && blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  launch_maybe_timed(take_launch_timer(), infer_mfma_kernel<T1, T2, FP8, MODE>, dim3(blocks), dim3(256), s, a);
}

template <int MODE>
int dispatch(const starnt_mlp& m, const InferArgs& a, hipStream_t s) {
  if (m.dtype == STARNT_F32) {
#define F32CASE(A, B) \
  if (m.h1 == A && m.h2 == B) { launch_f32<A, B, MODE>(a, s); return STARNT_OK; }
    F32CASE(16, 16) F32CASE(16, 32) F32CASE(32, 16) F32CASE(32, 32) F32CASE(32, 64) F32CASE(64, 32)
    F32CASE(64, 64) F32CASE(16, 64) F32CASE(64, 16)
#undef F32CASE
    return STARNT_EUNSUPPORTED;
  }
  if (m.dtype != STARNT_BF16 && m.dtype != STARNT_FP8) return STARNT_EUNSUPPORTED;
  const bool f8 = m.dtype == STARNT_FP8;
  const int t1 = (m.h1 + 31) / 32, t2 = (m.h2 + 31) / 32;
#define MCASE(A, B)                                                              \
  if (t1 == A && t2 == B) {                                                      \
    if (f8) launch_mfma<A, B, true, MODE>(a, s); else launch_mfma<A, B, false, MODE>(a, s); \
    return STARNT_OK;                                                            \
  }
  MCASE(1, 1) MCASE(1, 2) MCASE(2, 1) MCASE(2, 2)
#undef MCASE
  return STARNT_EUNSUPPORTED;
}

InferArgs make_args(const starnt_mlp& m, const float* tail, const uint32_t* count, const float* layer1,
                    const float* layer2, const float* tail_avg, const starnt_sched* sched, int W, int H,
                    const float* bg, float* out) {
  InferArgs a;
  a.W = W;
  a.H = H;
  a.tail = reinterpret_cast<const float4*>(tail);
  a.tail_avg = reinterpret_cast<const float4*>(tail_avg);
  a.level = nullptr;
  a.cs = 8;
  a.Cw = 1;
  a.count = count;
  a.layer1 = reinterpret_cast<const float4*>(layer1);
  a.layer2 = reinterpret_cast<const float4*>(layer2);
  a.sched = sched;
  a.W1 = m.W1; a.b1 = m.b1; a.W2 = m.W2; a.b2 = m.b2; a.W3 = m.W3; a.b3 = m.b3;
  a.in = m.in; a.h1 = m.h1; a.h2 = m.h2;
  for (int i = 0; i < 3; ++i) {
    a.sa[i] = m.fp8_scales ? m.fp8_scales[2 * i] : 1.0f;
    a.sw[i] = m.fp8_scales ? m.fp8_scales[2 * i + 1] : 1.0f;
  }
  a.bg0 = bg ? bg[0] : 0.0f;
  a.bg1 = bg ? bg[1] : 0.0f;
  a.bg2 = bg ? bg[2] : 0.0f;
  a.out = out;
  a.list = nullptr;
  a.list_n = nullptr;
  a.frame_p = 0;
  return a;
}

// the DFAOIT network input of every pixel, x [P][16] (zero where N < 3)
__global__ __launch_bounds__(256) void dfa_inputs_kernel(InferArgs a) {
  const int P = a.W * a.H;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const Grids g = load_grids(a.sched, a.W, a.H);
  PixIn in;
  load_pixel<kDfa>(a, g, p, in);
  float4* o = reinterpret_cast<float4*>(a.out) + 4 * (size_t)p;
  o[0] = make_float4(in.x[0], in.x[1], in.x[2], in.x[3]);
  o[1] = make_float4(in.x[4], in.x[5], in.x[6], in.x[7]);
  o[2] = make_float4(in.x[8], in.x[9], in.x[10], 0.0f);
  o[3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace

int launch_infer(const starnt_mlp& m, const float* tail, const uint32_t* count, const starnt_sched* sched,
                 int W, int H, float* out, hipStream_t s) {
  const InferArgs a = make_args(m, tail, count, nullptr, nullptr, nullptr, sched, W, H, nullptr, out);
  const int rc = dispatch<kTail>(m, a, s);
  if (rc) return fail(rc, "starnt_infer: unsupported dtype / hidden widths");
  STARNT_LAUNCH_CHECK("starnt_infer launch");
  return STARNT_OK;
}

int launch_infer_composite(const starnt_mlp& m, const starnt_feats& f, const starnt_sched* sched,
                           const float bg[3], float* rgb, hipStream_t s) {
  const InferArgs a = make_args(m, f.tail, f.count, f.layer1, f.layer2, f.tail_avg, sched, f.width, f.height, bg,
                                rgb);
  const int rc = m.variant == STARNT_NET_DFAOIT ? dispatch<kDfa>(m, a, s) : dispatch<kComp>(m, a, s);
  if (rc) return fail(rc, "starnt_infer_composite: unsupported dtype / hidden widths");
  STARNT_LAUNCH_CHECK("starnt_infer_composite launch");
  return STARNT_OK;
}

int launch_infer_composite_sel(const starnt_mlp& m, const starnt_feats& f, const starnt_sched* sched,
                               const uint8_t* level, int base, const float bg[3], float* rgb, hipStream_t s) {
  InferArgs a = make_args(m, f.tail, f.count, f.layer1, f.layer2, nullptr, sched, f.width, f.height, bg, rgb);
  a.level = level;
  a.cs = base / 8;
  a.Cw = (f.width + a.cs - 1) / a.cs;
  const int rc = dispatch<kSel>(m, a, s);
  if (rc) return fail(rc, "starnt_infer_composite_sel: unsupported dtype / hidden widths");
  STARNT_LAUNCH_CHECK("starnt_infer_composite_sel launch");
  return STARNT_OK;
}

int launch_infer_patch(const starnt_mlp& m, const starnt_feats& slots, const uint32_t* list,
                       const uint32_t* list_n, uint32_t frame_p, const float bg[3], float* rgb, hipStream_t s) {
  // the slots are a 1-row frame of `slots.width` pixels at full resolution
  InferArgs a = make_args(m, slots.tail, slots.count, slots.layer1, slots.layer2, nullptr, nullptr, slots.width, 1,
                          bg, rgb);
  a.list = list;
  a.list_n = list_n;
  a.frame_p = frame_p;
  const int rc = dispatch<kPatch>(m, a, s);
  if (rc) return fail(rc, "starnt_patch: unsupported dtype / hidden widths");
  STARNT_LAUNCH_CHECK("starnt_patch launch");
  return STARNT_OK;
}

int launch_dfa_inputs(const starnt_feats& f, const starnt_sched* sched, float* x, hipStream_t s) {
  starnt_mlp none{};
  const InferArgs a = make_args(none, f.tail, f.count, f.layer1, f.layer2, f.tail_avg, sched, f.width, f.height,
                                nullptr, x);
  const int P = f.width * f.height;
  hipLaunchKernelGGL(dfa_inputs_kernel, dim3((P + 255) / 256), dim3(256), 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_dfa_inputs launch");
  return STARNT_OK;
}

}  // namespace starnt
