// Passes 1-3 of STAR-NT (Sec. 3, Fig. 1) over per-pixel fragment lists.
//
// Per pixel:
//  * pass 1 (every pixel): nearest fragment by (depth, prim) -> d1, layer 1, N;
//  * pass 2 (pixels sampled by the pass-2 grid): second-nearest -> layer 2;
//  * pass 3 (pixels sampled by the pass-3 grid): order-independent sums over
//    ALL fragments in exact fixed point, then the two selected layers are
//    subtracted exactly, leaving the tail (sorted positions 3..N):
//      A = sum a, S = sum a c (a c rounded once in FP32), Lg = sum -log2(1 - a),
//    giving x = (N, t_tail = 2^-Lg, Ct = S / A) (Sec. 3.3).
// Integer sums make every output independent of the order of a list.
// Scales: A and S in Q24 (lane-local 32-bit partial sums, folded into 64 bits
// every 128 steps so they cannot overflow), Lg in Q27 in 64 bits; an opaque
// fragment (a = 1) adds 2^36 to Lg, so 2^-Lg is exactly 0 while it is in the
// tail and the exact subtraction removes it when it is a selected layer.
//
// Memory layout of the work: four lanes own a pixel and stride through its
// list together, so every load instruction of a quad covers a contiguous run
// of the CSR arrays (16 B of depth, 64 B of RGBA) that is consumed at once;
// a wave streams 16 neighbouring pixels, whose lists are adjacent in memory.
// No LDS and no barriers: the per-lane partial state (top-2 keys, 64-bit
// fixed-point sums) is merged across the quad with register shuffles.
#include "internal.h"

namespace starnt {
namespace {

constexpr float kQ24 = 16777216.0f;     // 2^24
constexpr float kQ27 = 134217728.0f;    // 2^27
constexpr uint64_t kOpaque = 1ull << 36;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kOne = 0x3F800000u;  // bits of 1.0f
constexpr int kG = 4;                   // lanes per pixel
constexpr uint32_t kFold = 128;         // lane steps between 32 -> 64-bit folds

struct FeatArgs {
  int W, H;
  const uint32_t* off;
  const float* depth;
  const void* rgba;
  const uint32_t* prim;
  uint32_t max_n;
  const starnt_sched* sched;
  float* d1;
  float4* layer1;
  uint32_t* count;
  float4* layer2;
  float4* tail;
  uint2* sel;
  uint32_t* err;
};

// Fixed-point terms of one fragment, rounded to nearest even (unbiased, so
// the error of a sum grows with the square root of its length). Each term is
// an exact integer function of its fragment, so the sums stay order
// independent.
struct Terms {
  uint32_t a, r, g, b;
  uint64_t lg;
};
__device__ __forceinline__ Terms frag_terms(float4 c) {
  Terms t;
  const float a = __builtin_amdgcn_fmed3f(c.w, 0.0f, 1.0f);
  const float a24 = a * kQ24;  // exact scaling: a24 * c = (a * c) * 2^24
  t.a = (uint32_t)__builtin_rintf(a24);
  t.r = (uint32_t)__builtin_rintf(a24 * c.x);
  t.g = (uint32_t)__builtin_rintf(a24 * c.y);
  t.b = (uint32_t)__builtin_rintf(a24 * c.z);
  const float l = -__log2f(1.0f - a) * kQ27;  // <= 24 * 2^27 below a = 1
  t.lg = a >= 1.0f ? kOpaque : (uint64_t)(uint32_t)__builtin_rintf(l);
  return t;
}

// pixel totals (64-bit) and the lane-local 32-bit partials
struct Sums {
  uint64_t a = 0, r = 0, g = 0, b = 0, lg = 0;
};
struct Part {
  uint32_t a = 0, r = 0, g = 0, b = 0;
};
__device__ __forceinline__ void fold(Sums& s, Part& p) {
  s.a += p.a; s.r += p.r; s.g += p.g; s.b += p.b;
  p = Part();
}

// two smallest (depth, prim) keys; prim is read only on equal depths
struct Top2 {
  float z1 = __builtin_inff(), z2 = __builtin_inff();
  uint32_t k1 = kNone, k2 = kNone;  // global fragment indices
};

__device__ __forceinline__ bool key_less(float z, uint32_t k, float zb, uint32_t kb, const uint32_t* prim) {
  if (z < zb) return true;
  if (z > zb || kb == kNone) return false;
  if (z != zb) return false;  // NaN
  return prim[k] < prim[kb];
}

__device__ __forceinline__ void top2_push(Top2& t, float z, uint32_t k, const uint32_t* prim) {
  if (key_less(z, k, t.z1, t.k1, prim)) {
    t.z2 = t.z1; t.k2 = t.k1;
    t.z1 = z; t.k1 = k;
  } else if (key_less(z, k, t.z2, t.k2, prim)) {
    t.z2 = z; t.k2 = k;
  }
}

template <bool HALF, bool RGBA>
__device__ __forceinline__ void step(const FeatArgs& a, uint32_t k, Top2& t, Part& p, Sums& s, uint32_t& zmax,
                                     uint32_t& amax) {
  const float z = a.depth[k];
  zmax = max(zmax, __float_as_uint(z));  // -0, negatives and NaN exceed 1.0's bits
  top2_push(t, z, k, a.prim);
  if constexpr (RGBA) {
    const float4 c = load_rgba<HALF>(a.rgba, k);
    amax = max(amax, __float_as_uint(c.w));
    const Terms q = frag_terms(c);
    p.a += q.a; p.r += q.r; p.g += q.g; p.b += q.b;
    s.lg += q.lg;
  }
}

// one lane's share of a list: fragments b+q, b+q+4, ... two per step so both
// loads are in flight together; 32-bit partials folded every kFold steps
template <bool HALF, bool RGBA>
__device__ __forceinline__ void stream(const FeatArgs& a, uint32_t b, uint32_t e, int q, Top2& t, Sums& s,
                                       uint32_t& zmax, uint32_t& amax) {
  Part p;
  uint32_t k = b + q;
  while (k < e) {
    const uint32_t kend = min(e, k + kFold * kG);
    for (; k + kG < kend; k += 2 * kG) {
      const float z0 = a.depth[k], z1 = a.depth[k + kG];
      float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
      if constexpr (RGBA) {
        c0 = load_rgba<HALF>(a.rgba, k);
        c1 = load_rgba<HALF>(a.rgba, k + kG);
      }
      zmax = max(zmax, max(__float_as_uint(z0), __float_as_uint(z1)));
      top2_push(t, z0, k, a.prim);
      top2_push(t, z1, k + kG, a.prim);
      if constexpr (RGBA) {
        amax = max(amax, max(__float_as_uint(c0.w), __float_as_uint(c1.w)));
        const Terms q0 = frag_terms(c0), q1 = frag_terms(c1);
        p.a += q0.a + q1.a; p.r += q0.r + q1.r; p.g += q0.g + q1.g; p.b += q0.b + q1.b;
        s.lg += q0.lg + q1.lg;
      }
    }
    if (k < kend) {
      step<HALF, RGBA>(a, k, t, p, s, zmax, amax);
      k += kG;
    }
    fold(s, p);
  }
}

template <bool HALF>
__global__ __launch_bounds__(256) void features_kernel(FeatArgs a) {
  const int P = a.W * a.H;
  const int q = threadIdx.x & (kG - 1);
  const int p = (int)((blockIdx.x * (unsigned)blockDim.x + threadIdx.x) / kG);
  if (p >= P) return;  // whole quads leave together
  const Grids g = load_grids(a.sched, a.W, a.H);
  const int x = p % a.W, y = p / a.W;
  const int i2 = grid_index_of(x, a.W, g.w2), j2 = grid_index_of(y, a.H, g.h2);
  const int i3 = grid_index_of(x, a.W, g.w3), j3 = grid_index_of(y, a.H, g.h3);
  const bool pass2 = i2 >= 0 && j2 >= 0;
  const bool pass3 = i3 >= 0 && j3 >= 0;

  const uint32_t b = a.off[p], e = a.off[p + 1];
  const uint32_t n = e - b;
  Top2 t;
  Sums s;
  uint32_t zmax = 0, amax = 0;
  if (pass3) stream<HALF, true>(a, b, e, q, t, s, zmax, amax);
  else stream<HALF, false>(a, b, e, q, t, s, zmax, amax);

  // merge the quad: two xor-shuffle rounds
#pragma unroll
  for (int m = 1; m < kG; m <<= 1) {
    const float oz1 = __shfl_xor(t.z1, m), oz2 = __shfl_xor(t.z2, m);
    const uint32_t ok1 = __shfl_xor(t.k1, m), ok2 = __shfl_xor(t.k2, m);
    top2_push(t, oz1, ok1, a.prim);
    top2_push(t, oz2, ok2, a.prim);
    if (pass3) {
      s.a += __shfl_xor(s.a, m);
      s.r += __shfl_xor(s.r, m);
      s.g += __shfl_xor(s.g, m);
      s.b += __shfl_xor(s.b, m);
      s.lg += __shfl_xor(s.lg, m);
    }
  }
  // the two selected layers: lane 0 fetches layer 1, lane 1 layer 2, and the
  // quad shares them
  const bool want2 = pass2 || pass3;
  float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
  if (q == 0 && t.k1 != kNone) c = load_rgba<HALF>(a.rgba, t.k1);
  if (q == 1 && t.k2 != kNone && want2) c = load_rgba<HALF>(a.rgba, t.k2);
  const int base = threadIdx.x & ~(kG - 1);
  const float4 c1 = make_float4(__shfl(c.x, base), __shfl(c.y, base), __shfl(c.z, base), __shfl(c.w, base));
  const float4 c2 = make_float4(__shfl(c.x, base + 1), __shfl(c.y, base + 1), __shfl(c.z, base + 1),
                                __shfl(c.w, base + 1));
  // outputs, spread over the quad
  if (q == 0) {
    const float a1 = __builtin_amdgcn_fmed3f(c1.w, 0.0f, 1.0f);
    a.d1[p] = n ? t.z1 : 1.0f;
    a.layer1[p] = make_float4(a1 * c1.x, a1 * c1.y, a1 * c1.z, a1);
    a.count[p] = n;
    if (a.sel) a.sel[p] = make_uint2(t.k1, t.k2);
  } else if (q == 1 && pass2) {
    const float a2 = __builtin_amdgcn_fmed3f(c2.w, 0.0f, 1.0f);
    a.layer2[j2 * g.w2 + i2] = make_float4(a2 * c2.x, a2 * c2.y, a2 * c2.z, a2);
  } else if (q >= 2 && pass3) {
    // exact removal of the two selected layers leaves the tail
    if (t.k1 != kNone) {
      const Terms r = frag_terms(c1);
      s.a -= r.a; s.r -= r.r; s.g -= r.g; s.b -= r.b; s.lg -= r.lg;
    }
    if (t.k2 != kNone) {
      const Terms r = frag_terms(c2);
      s.a -= r.a; s.r -= r.r; s.g -= r.g; s.b -= r.b; s.lg -= r.lg;
    }
    float4* o = a.tail + 2 * (size_t)(j3 * g.w3 + i3);
    const bool tail = n > 2;
    const float inv = (tail && s.a) ? 1.0f / (float)s.a : 0.0f;
    if (q == 2) {
      const float tt = tail ? exp2f(-(float)s.lg * (1.0f / kQ27)) : 1.0f;
      o[0] = make_float4((float)n, tt, (float)s.r * inv, (float)s.g * inv);
    } else {
      o[1] = make_float4((float)s.b * inv, tail ? (float)s.a * (1.0f / kQ24) : 0.0f, 0.0f, 0.0f);
    }
  }
  uint32_t errf = (q == 0 && n > a.max_n) ? STARNT_DERR_COUNT : 0u;
  errf |= zmax > kOne ? STARNT_DERR_DEPTH : 0u;
  errf |= amax > kOne ? STARNT_DERR_ALPHA : 0u;
  if (errf) atomicOr(a.err, errf);
}

}  // namespace

int launch_features(const starnt_frags& f, const starnt_sched* sched, const starnt_feats& o, hipStream_t s) {
  FeatArgs a;
  a.W = f.width;
  a.H = f.height;
  a.off = f.offsets;
  a.depth = f.depth;
  a.rgba = f.rgba;
  a.prim = f.prim;
  a.max_n = f.max_per_pixel;
  a.sched = sched;
  a.d1 = o.d1;
  a.layer1 = reinterpret_cast<float4*>(o.layer1);
  a.count = o.count;
  a.layer2 = reinterpret_cast<float4*>(o.layer2);
  a.tail = reinterpret_cast<float4*>(o.tail);
  a.sel = reinterpret_cast<uint2*>(o.sel);
  a.err = o.err;
  const int P = f.width * f.height;
  const dim3 block(256), grid((unsigned)(((int64_t)P * kG + 255) / 256));
  if (f.rgba_dtype == STARNT_F16)
    hipLaunchKernelGGL(features_kernel<true>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(features_kernel<false>, grid, block, 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_features launch");
  return STARNT_OK;
}

}  // namespace starnt
