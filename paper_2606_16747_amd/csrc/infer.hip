// Tail-colour network f(x) of STAR-NT (Sec. 3.3) at full resolution, over the
// bilinearly upscaled pass-3 features (Sec. 3.2). Three dense layers with ReLU
// after each; x = (N, t_tail, Ct_rgb) plus zero padding to 16 inputs.
//
// Paths:
//  * STARNT_F32  : one thread per pixel, FP32 FMAs, weights read with
//                  wave-uniform addresses (scalar loads).
//  * STARNT_BF16 : matrix cores. Pixels are the N dimension of
//                  v_mfma_f32_32x32x16_bf16 (32 pixels per wave step); a layer
//                  is H^T = W H_prev^T. The hidden units of layer 1 are stored
//                  in a permuted order chosen so that each lane's accumulator
//                  registers of layer 1 are exactly its B-operand registers of
//                  layer 2: no data moves between lanes. The 3-wide output
//                  layer runs on the VALU from bf16-rounded operands.
//  * STARNT_FP8  : the same structure with E4M3 operands and per-layer scales
//                  (v_mfma_f32_32x32x64_f8f6f4 is not needed: K = 16 per step
//                  uses v_mfma_f32_32x32x16_fp8_fp8).
#include "internal.h"

namespace starnt {
namespace {

struct InferArgs {
  int W, H;
  const float4* tail;
  const uint32_t* count;
  const starnt_sched* sched;
  const float* __restrict__ W1;
  const float* __restrict__ b1;
  const float* __restrict__ W2;
  const float* __restrict__ b2;
  const float* __restrict__ W3;
  const float* __restrict__ b3;
  int in, h1, h2;
  float sa[3], sw[3];  // FP8 scales
  float* out;
};

// upscaled features x0..x4 of full-resolution pixel (x, y)
__device__ __forceinline__ void fetch_x(const InferArgs& a, const Grids& g, int x, int y, float v[5]) {
  const Taps tx = axis_taps(x, a.W, g.w3), ty = axis_taps(y, a.H, g.h3);
  const size_t i00 = (size_t)ty.i0 * g.w3 + tx.i0, i01 = (size_t)ty.i0 * g.w3 + tx.i1;
  const size_t i10 = (size_t)ty.i1 * g.w3 + tx.i0, i11 = (size_t)ty.i1 * g.w3 + tx.i1;
  const float4 a00 = a.tail[2 * i00], c00 = a.tail[2 * i00 + 1];
  float4 r0 = a00;
  float r4 = c00.x;
  if (tx.w1 != 0.0f || ty.w1 != 0.0f) {
    const float4 a01 = a.tail[2 * i01], c01 = a.tail[2 * i01 + 1];
    const float4 a10 = a.tail[2 * i10], c10 = a.tail[2 * i10 + 1];
    const float4 a11 = a.tail[2 * i11], c11 = a.tail[2 * i11 + 1];
    const float wx = tx.w1, wy = ty.w1;
    auto l = [](float p, float q, float w) { return fmaf(w, q - p, p); };
    r0.x = l(l(a00.x, a01.x, wx), l(a10.x, a11.x, wx), wy);
    r0.y = l(l(a00.y, a01.y, wx), l(a10.y, a11.y, wx), wy);
    r0.z = l(l(a00.z, a01.z, wx), l(a10.z, a11.z, wx), wy);
    r0.w = l(l(a00.w, a01.w, wx), l(a10.w, a11.w, wx), wy);
    r4 = l(l(c00.x, c01.x, wx), l(c10.x, c11.x, wx), wy);
  }
  v[0] = r0.x; v[1] = r0.y; v[2] = r0.z; v[3] = r0.w; v[4] = r4;
}

// ---------------------------------------------------------------------------
// FP32 VALU path

template <int H1, int H2>
__global__ __launch_bounds__(256) void infer_f32_kernel(InferArgs a) {
  const int P = a.W * a.H;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const uint32_t n = a.count[p];
  float o0 = 0.f, o1 = 0.f, o2 = 0.f;
  if (n >= 3) {
    const Grids g = load_grids(a.sched, a.W, a.H);
    float x[5];
    fetch_x(a, g, p % a.W, p / a.W, x);
    float h1[H1];
#pragma unroll
    for (int j = 0; j < H1; ++j) {
      float s = a.b1[j];
#pragma unroll
      for (int i = 0; i < 5; ++i) s = fmaf(a.W1[j * a.in + i], x[i], s);
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
    o0 = fmaxf(s0, 0.0f);
    o1 = fmaxf(s1, 0.0f);
    o2 = fmaxf(s2, 0.0f);
  }
  a.out[3 * (size_t)p + 0] = o0;
  a.out[3 * (size_t)p + 1] = o1;
  a.out[3 * (size_t)p + 2] = o2;
}

// ---------------------------------------------------------------------------
// BF16 matrix-core path

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ __bf16 to_bf16(float v) { return static_cast<__bf16>(v); }
__device__ __forceinline__ float bf16_round(float v) { return static_cast<float>(static_cast<__bf16>(v)); }

// Physical accumulator row r of a 32-row tile (lane half h = (r % 8) / 4,
// block b = r / 8, element i = r % 4) holds logical hidden unit
// 16 (b / 2) + 8 h + 4 (b % 2) + i, so that accumulator register v = 4 b + i
// of lane half h is element (v % 8) of B-operand chunk (v / 8) for the next
// layer (chunk K index 8 h + e).
__device__ __forceinline__ int perm_row(int r) {
  const int b = r >> 3, h = (r >> 2) & 1, i = r & 3;
  return 16 * (b >> 1) + 8 * h + 4 * (b & 1) + i;
}

// T1, T2: number of 32-row tiles of the two hidden layers (h padded with zero
// weights up to 32 * T).
template <int T1, int T2>
__global__ __launch_bounds__(256) void infer_bf16_kernel(InferArgs a) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int waves_per_block = blockDim.x >> 6;
  const int wave = blockIdx.x * waves_per_block + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * waves_per_block;
  const int P = a.W * a.H;
  const int ngroups = (P + 31) / 32;
  const Grids g = load_grids(a.sched, a.W, a.H);

  // ---- weights into registers, in operand layout ----
  // layer 1 A operand: tile t, physical row `col`, inputs 8*half .. 8*half+7
  bf16x8 A1[T1];
  f32x16 B1v[T1];  // bias per accumulator register
#pragma unroll
  for (int t = 0; t < T1; ++t) {
    const int u = 32 * t + perm_row(col);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * half + e;
      const float w = (u < a.h1 && k < 5) ? a.W1[u * a.in + k] : 0.0f;
      A1[t][e] = to_bf16(w);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v >> 2) + 4 * half + (v & 3);
      const int uu = 32 * t + perm_row(r);
      B1v[t][v] = uu < a.h1 ? a.b1[uu] : 0.0f;
    }
  }
  // layer 2 A operand: tile t2 (rows = h2 units 32 t2 + col), K chunk c over
  // logical h1 units 16 c + 8 half + e
  constexpr int C2 = 2 * T1;
  bf16x8 A2[T2][C2];
  f32x16 B2v[T2];
#pragma unroll
  for (int t = 0; t < T2; ++t) {
    const int row = 32 * t + col;
#pragma unroll
    for (int c = 0; c < C2; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * c + 8 * half + e;
        const float w = (row < a.h2 && k < a.h1) ? a.W2[row * a.h1 + k] : 0.0f;
        A2[t][c][e] = to_bf16(w);
      }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 32 * t + 8 * (v >> 2) + 4 * half + (v & 3);
      B2v[t][v] = r < a.h2 ? a.b2[r] : 0.0f;
    }
  }
  // output layer (VALU) weights for this lane's h2 rows, bf16-rounded
  float W3v[3][T2][16];
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int t = 0; t < T2; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = 32 * t + 8 * (v >> 2) + 4 * half + (v & 3);
        W3v[o][t][v] = r < a.h2 ? bf16_round(a.W3[o * a.h2 + r]) : 0.0f;
      }
  const float b30 = a.b3[0], b31 = a.b3[1], b32 = a.b3[2];

  for (int grp = wave; grp < ngroups; grp += nwaves) {
    const int p = grp * 32 + col;
    const bool live = p < P;
    const uint32_t n = live ? a.count[p] : 0u;
    // B operand of layer 1: inputs 8 half .. 8 half + 7 of pixel p
    bf16x8 X;
#pragma unroll
    for (int e = 0; e < 8; ++e) X[e] = to_bf16(0.0f);
    if (half == 0 && n >= 3) {
      float v[5];
      fetch_x(a, g, p % a.W, p / a.W, v);
#pragma unroll
      for (int e = 0; e < 5; ++e) X[e] = to_bf16(v[e]);
    }
    // layer 1
    bf16x8 Hb[C2];
#pragma unroll
    for (int t = 0; t < T1; ++t) {
      f32x16 acc = B1v[t];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[t], X, acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) Hb[2 * t + (v >> 3)][v & 7] = to_bf16(fmaxf(acc[v], 0.0f));
    }
    // layer 2 + output layer
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int t = 0; t < T2; ++t) {
      f32x16 acc = B2v[t];
#pragma unroll
      for (int c = 0; c < C2; ++c) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A2[t][c], Hb[c], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float h = bf16_round(fmaxf(acc[v], 0.0f));
        s0 = fmaf(W3v[0][t][v], h, s0);
        s1 = fmaf(W3v[1][t][v], h, s1);
        s2 = fmaf(W3v[2][t][v], h, s2);
      }
    }
    // the two lane halves hold the two halves of the h2 rows of pixel p
    s0 += __shfl_xor(s0, 32);
    s1 += __shfl_xor(s1, 32);
    s2 += __shfl_xor(s2, 32);
    if (half == 0 && live) {
      const bool on = n >= 3;
      a.out[3 * (size_t)p + 0] = on ? fmaxf(s0 + b30, 0.0f) : 0.0f;
      a.out[3 * (size_t)p + 1] = on ? fmaxf(s1 + b31, 0.0f) : 0.0f;
      a.out[3 * (size_t)p + 2] = on ? fmaxf(s2 + b32, 0.0f) : 0.0f;
    }
  }
}

template <int H1, int H2>
int launch_f32(const InferArgs& a, hipStream_t s) {
  const int P = a.W * a.H;
  hipLaunchKernelGGL((infer_f32_kernel<H1, H2>), dim3((P + 255) / 256), dim3(256), 0, s, a);
  return STARNT_OK;
}

template <int T1, int T2>
int launch_bf16(const InferArgs& a, hipStream_t s) {
  const int P = a.W * a.H;
  const int groups = (P + 31) / 32;
  // persistent waves: enough to fill the chip, each walking many 32-pixel groups
  int blocks = (groups + 3) / 4;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((infer_bf16_kernel<T1, T2>), dim3(blocks), dim3(256), 0, s, a);
  return STARNT_OK;
}

}  // namespace

int launch_infer(const starnt_mlp& m, const float* tail, const uint32_t* count, const starnt_sched* sched,
                 int W, int H, float* out, hipStream_t s) {
  InferArgs a;
  a.W = W;
  a.H = H;
  a.tail = reinterpret_cast<const float4*>(tail);
  a.count = count;
  a.sched = sched;
  a.W1 = m.W1; a.b1 = m.b1; a.W2 = m.W2; a.b2 = m.b2; a.W3 = m.W3; a.b3 = m.b3;
  a.in = m.in; a.h1 = m.h1; a.h2 = m.h2;
  for (int i = 0; i < 3; ++i) {
    a.sa[i] = m.fp8_scales ? m.fp8_scales[2 * i] : 1.0f;
    a.sw[i] = m.fp8_scales ? m.fp8_scales[2 * i + 1] : 1.0f;
  }
  a.out = out;
  int rc = STARNT_EUNSUPPORTED;
  if (m.dtype == STARNT_F32) {
#define F32CASE(A, B) \
  if (m.h1 == A && m.h2 == B) rc = launch_f32<A, B>(a, s);
    F32CASE(16, 16) F32CASE(16, 32) F32CASE(32, 16) F32CASE(32, 32) F32CASE(32, 64) F32CASE(64, 32)
    F32CASE(64, 64) F32CASE(16, 64) F32CASE(64, 16)
#undef F32CASE
  } else if (m.dtype == STARNT_BF16) {
    const int t1 = (m.h1 + 31) / 32, t2 = (m.h2 + 31) / 32;
    if (t1 == 1 && t2 == 1) rc = launch_bf16<1, 1>(a, s);
    else if (t1 == 1 && t2 == 2) rc = launch_bf16<1, 2>(a, s);
    else if (t1 == 2 && t2 == 1) rc = launch_bf16<2, 1>(a, s);
    else if (t1 == 2 && t2 == 2) rc = launch_bf16<2, 2>(a, s);
  }
  if (rc == STARNT_EUNSUPPORTED) return fail(rc, "starnt_infer: unsupported dtype / hidden widths");
  STARNT_LAUNCH_CHECK("starnt_infer launch");
  return rc;
}

}  // namespace starnt
