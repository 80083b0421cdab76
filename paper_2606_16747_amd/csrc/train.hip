// Training step of the tail-colour network (Sec. 3.3: MSE loss, Adam), on the
// GPU with FP32 master weights. The loss may weight each sample's squared
// error (the composite-space error takes T2^2, since eq (3) scales f by T2).
//
// Kernel 1: one block per slice of kSB samples. Forward and backward run with
//   the slice's activations in LDS; the block writes its partial loss and its
//   partial gradient (sum over its samples) for every parameter.
// Kernel 2: sums the partials of every parameter in a fixed order (so a step
//   is bitwise reproducible), then applies bias-corrected Adam to the FP32
//   master weight.
// In BF16 mode every GEMM operand (weights, inputs, activations, output
// gradients) is rounded to bf16 as the matrix cores would consume it; products
// of two bf16 values are exact in FP32 and accumulation is FP32.
// In FP8 mode the three forward products take OCP E4M3 operands on
// v_mfma_f32_32x32x16_fp8_fp8: weights with a per-layer power-of-two scale
// from the masters' largest magnitude, inputs and activations with the
// caller's per-layer power-of-two scales. The backward products and weight
// gradients run in bf16 on those same E4M3 values (a power-of-two multiple
// of an E4M3 value is exact in bf16) and on bf16 output gradients, so the
// gradient is that of the FP8 forward pass.
//
// BF16 with hidden widths 32 or 64 runs kernel 1 on the matrix cores
// (train_mfma_kernel, below); FP32 and other widths use train_fwd_bwd on the
// vector units. Both take the same rounding points.
#include <cmath>

#include "internal.h"

namespace starnt {
namespace {

constexpr int kSB = 64;    // samples per block
constexpr int kIn = 16;

struct TrainArgs {
  int batch, h1, h2;
  const float* params;
  const float* x;
  const float* y;
  const float* wt;      // [batch] per-sample loss weights (NULL: 1)
  float* partial;       // [nblocks][nparam]
  float* partial_loss;  // [nblocks]
  int nparam;
  float inv_count;      // 1 / (batch * 3)
  int out_act;          // 0 ReLU, 1 logistic sigmoid
  float sa[3];          // FP8: activation scale of each layer's input (powers of two)
};

template <bool BF>
__device__ __forceinline__ float q(float v) {
  if constexpr (BF) return static_cast<float>(static_cast<__bf16>(v));
  else return v;
}

template <bool BF, int H1, int H2>
__global__ __launch_bounds__(256) void train_fwd_bwd(TrainArgs a) {
  __shared__ float s_x[kSB][kIn];
  __shared__ float s_h1[kSB][H1];   // relu(z1) (bf16-rounded in BF16 mode)
  __shared__ float s_h2[kSB][H2];
  __shared__ float s_d1[kSB][H1];
  __shared__ float s_d2[kSB][H2];
  __shared__ float s_d3[kSB][4];
  __shared__ float s_loss[256];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kSB;
  const int ns = min(kSB, a.batch - s0);
  const float* W1 = a.params;
  const float* b1 = W1 + H1 * kIn;
  const float* W2 = b1 + H1;
  const float* b2 = W2 + H2 * H1;
  const float* W3 = b2 + H2;
  const float* b3 = W3 + 3 * H2;

  for (int i = tid; i < kSB * kIn; i += 256) {
    const int s = i / kIn, c = i % kIn;
    s_x[s][c] = s < ns ? q<BF>(a.x[(size_t)(s0 + s) * kIn + c]) : 0.0f;
  }
  __syncthreads();
  // layer 1
  for (int i = tid; i < kSB * H1; i += 256) {
    const int s = i / H1, j = i % H1;
    float z = b1[j];
    for (int c = 0; c < kIn; ++c) z = fmaf(q<BF>(W1[j * kIn + c]), s_x[s][c], z);
    s_h1[s][j] = z > 0.0f ? q<BF>(z) : 0.0f;
    s_d1[s][j] = z > 0.0f ? 1.0f : 0.0f;   // ReLU mask, reused below
  }
  __syncthreads();
  // layer 2
  for (int i = tid; i < kSB * H2; i += 256) {
    const int s = i / H2, k = i % H2;
    float z = b2[k];
    for (int j = 0; j < H1; ++j) z = fmaf(q<BF>(W2[k * H1 + j]), s_h1[s][j], z);
    s_h2[s][k] = z > 0.0f ? q<BF>(z) : 0.0f;
    s_d2[s][k] = z > 0.0f ? 1.0f : 0.0f;
  }
  __syncthreads();
  // output layer and loss
  float lsum = 0.0f;
  for (int i = tid; i < kSB * 3; i += 256) {
    const int s = i / 3, o = i % 3;
    float d = 0.0f;
    if (s < ns) {
      float z = b3[o];
      for (int k = 0; k < H2; ++k) z = fmaf(q<BF>(W3[o * H2 + k]), s_h2[s][k], z);
      const float f = a.out_act ? 1.0f / (1.0f + expf(-z)) : fmaxf(z, 0.0f);
      const float e = f - a.y[(size_t)(s0 + s) * 3 + o];
      const float wk = a.wt ? a.wt[s0 + s] : 1.0f;
      lsum = fmaf(wk * e * e, a.inv_count, lsum);
      const float df = a.out_act ? f * (1.0f - f) : (z > 0.0f ? 1.0f : 0.0f);
      d = 2.0f * wk * e * a.inv_count * df;
    }
    s_d3[s][o] = q<BF>(d);
  }
  s_loss[tid] = lsum;
  __syncthreads();
  // dL/dz2
  for (int i = tid; i < kSB * H2; i += 256) {
    const int s = i / H2, k = i % H2;
    float g = 0.0f;
    for (int o = 0; o < 3; ++o) g = fmaf(q<BF>(W3[o * H2 + k]), s_d3[s][o], g);
    s_d2[s][k] = q<BF>(g * s_d2[s][k]);
  }
  __syncthreads();
  // dL/dz1
  for (int i = tid; i < kSB * H1; i += 256) {
    const int s = i / H1, j = i % H1;
    float g = 0.0f;
    for (int k = 0; k < H2; ++k) g = fmaf(q<BF>(W2[k * H1 + j]), s_d2[s][k], g);
    s_d1[s][j] = q<BF>(g * s_d1[s][j]);
  }
  __syncthreads();
  // partial gradients of this block, one parameter per thread-iteration
  float* out = a.partial + (size_t)blockIdx.x * a.nparam;
  const int n1 = H1 * kIn, n2 = n1 + H1, n3 = n2 + H2 * H1, n4 = n3 + H2, n5 = n4 + 3 * H2;
  for (int i = tid; i < a.nparam; i += 256) {
    float g = 0.0f;
    if (i < n1) {
      const int j = i / kIn, c = i % kIn;
      for (int s = 0; s < kSB; ++s) g = fmaf(s_d1[s][j], s_x[s][c], g);
    } else if (i < n2) {
      const int j = i - n1;
      for (int s = 0; s < kSB; ++s) g += s_d1[s][j];
    } else if (i < n3) {
      const int k = (i - n2) / H1, j = (i - n2) % H1;
      for (int s = 0; s < kSB; ++s) g = fmaf(s_d2[s][k], s_h1[s][j], g);
    } else if (i < n4) {
      const int k = i - n3;
      for (int s = 0; s < kSB; ++s) g += s_d2[s][k];
    } else if (i < n5) {
      const int o = (i - n4) / H2, k = (i - n4) % H2;
      for (int s = 0; s < kSB; ++s) g = fmaf(s_d3[s][o], s_h2[s][k], g);
    } else {
      const int o = i - n5;
      for (int s = 0; s < kSB; ++s) g += s_d3[s][o];
    }
    out[i] = g;
  }
  // block loss: fixed-order tree
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) s_loss[tid] += s_loss[tid + w];
    __syncthreads();
  }
  if (tid == 0) a.partial_loss[blockIdx.x] = s_loss[0];
}

struct AdamArgs {
  int nparam, nblocks;
  const float* partial;
  const float* partial_loss;
  float* params;
  float* m;
  float* v;
  float* grad;
  float* loss;
  float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
};

// 16 parameters x 16 row groups per block: thread (r, c) sums the partials
// of rows r, r + 16, ... for parameter c; the 16 group sums are then added in
// order. The order is fixed, so the gradient is bitwise reproducible.
constexpr int kRP = 16;   // parameters per block
constexpr int kRG = 16;   // row groups per block

__global__ __launch_bounds__(kRP * kRG) void train_reduce_adam(AdamArgs a) {
  __shared__ float s_part[kRG][kRP];
  const int c = threadIdx.x % kRP, r = threadIdx.x / kRP;
  const int i = blockIdx.x * kRP + c;
  float g = 0.0f;
  if (i < a.nparam) {
    // four loads in flight per step, added in the same order as one by one
    int b = r;
    for (; b + 3 * kRG < a.nblocks; b += 4 * kRG) {
      const float p0 = a.partial[(size_t)b * a.nparam + i];
      const float p1 = a.partial[(size_t)(b + kRG) * a.nparam + i];
      const float p2 = a.partial[(size_t)(b + 2 * kRG) * a.nparam + i];
      const float p3 = a.partial[(size_t)(b + 3 * kRG) * a.nparam + i];
      g += p0;
      g += p1;
      g += p2;
      g += p3;
    }
    for (; b < a.nblocks; b += kRG) g += a.partial[(size_t)b * a.nparam + i];
  }
  s_part[r][c] = g;
  // the optimiser state is read before any store (a store ahead of a load
  // from a pointer that might alias it would wait for the load)
  float m0 = 0.0f, v0 = 0.0f, w0 = 0.0f;
  if (r == 0 && i < a.nparam) {
    m0 = a.m[i];
    v0 = a.v[i];
    w0 = a.params[i];
  }
  __syncthreads();
  if (r == 0 && i < a.nparam) {
    float t = 0.0f;
    for (int k = 0; k < kRG; ++k) t += s_part[k][c];
    const float m = fmaf(a.b1, m0, (1.0f - a.b1) * t);
    const float v = fmaf(a.b2, v0, (1.0f - a.b2) * t * t);
    const float mh = m / a.c1, vh = v / a.c2;
    a.grad[i] = t;
    a.m[i] = m;
    a.v[i] = v;
    a.params[i] = w0 - a.lr * mh / (sqrtf(vh) + a.eps);
  }
  if (blockIdx.x == 0) {
    // loss: per-thread strided sums, then a fixed-order tree
    __shared__ float s_loss[kRP * kRG];
    float l = 0.0f;
    for (int b = threadIdx.x; b < a.nblocks; b += kRP * kRG) l += a.partial_loss[b];
    s_loss[threadIdx.x] = l;
    __syncthreads();
    for (int w = kRP * kRG / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s_loss[threadIdx.x] += s_loss[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.loss[0] = s_loss[0];
  }
}

// ---------------------------------------------------------------------------
// Kernel 1 on the matrix cores (BF16, h1 and h2 in {32, 64}).
//
// A block is 4 waves and kMSamples = 256 samples; wave w owns samples
// 64 w .. 64 w + 63 as two 32-sample groups (the N dimension of
// v_mfma_f32_32x32x16_bf16).
//  * Per group, in registers: the forward pass, dL/dz3, dL/dh2 = W3^T dz3 and
//    dL/dh1 = W2^T dz2. Hidden rows are stored permuted (perm_row), so each
//    product's accumulators are already the next product's B operand.
//  * The weight gradients contract over samples. x, h1, h2 and dz1..dz3 of all
//    256 samples are staged in LDS as [unit][sample] bf16 rows; after one
//    barrier the waves share out the gradient tiles, each a product with
//    K = 256 samples whose result is final for the block and goes straight to
//    the block's partial. Bias gradients are fixed-order row sums, one row
//    per thread. train_reduce_adam then sums the blocks' partials in order.

constexpr int kMWaves = 4;
constexpr int kMSamples = 64 * kMWaves;      // samples per block
constexpr int kRow = kMSamples + 8;          // LDS row stride in bf16 (offsets rows by 4 banks)

__device__ __forceinline__ f32x16 mfma_bf16(const bf16x8& A, const bf16x8& B, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 pack8(const float* w) {
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = static_cast<__bf16>(w[e]);
  return v;
}

// 8 consecutive bf16 of an LDS row (16-byte aligned)
__device__ __forceinline__ bf16x8 lds8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Forward-pass operands: bf16, or E4M3 bytes of v * inv_s (FP8; every value
// is already an E4M3 value times the scale, so the convert is exact)
template <bool FP8>
using FwdVec = typename std::conditional<FP8, fp8x8, bf16x8>::type;
template <bool FP8>
__device__ __forceinline__ FwdVec<FP8> pack_fwd(const float* w, float inv_s) {
  if constexpr (FP8) {
    const uint32_t lo = e4m3_pack4(sat448(w[0] * inv_s), sat448(w[1] * inv_s), sat448(w[2] * inv_s),
                                   sat448(w[3] * inv_s));
    const uint32_t hi = e4m3_pack4(sat448(w[4] * inv_s), sat448(w[5] * inv_s), sat448(w[6] * inv_s),
                                   sat448(w[7] * inv_s));
    return (long)(((unsigned long)hi << 32) | lo);
  } else {
    return pack8(w);
  }
}
template <bool FP8>
__device__ __forceinline__ f32x16 mfma_fwd(const FwdVec<FP8>& A, const FwdVec<FP8>& B, f32x16 c) {
  if constexpr (FP8) return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(A, B, c, 0, 0, 0);
  else return mfma_bf16(A, B, c);
}
// The operand value a forward product sees: v rounded to bf16, or (FP8) to
// the E4M3 grid of scale s (a power of two, so the result is also exact in
// bf16 and the backward products and weight gradients take the same value)
template <bool FP8>
__device__ __forceinline__ float fwd_value(float v, float s, float inv_s) {
  if constexpr (FP8) return e4m3_value(v * inv_s) * s;
  else return q<true>(v);
}
// smallest power of two s with amax / s <= 448 (1 when amax is 0), by exact
// comparisons on the exponent of amax
__device__ __forceinline__ float e4m3_scale_for(float amax) {
  if (!(amax > 0.0f)) return 1.0f;
  int e;
  const float m = frexpf(amax, &e);  // amax = m 2^e, m in [0.5, 1); 448 = 0.875 2^9
  return ldexpf(1.0f, m <= 0.875f ? e - 9 : e - 8);
}

template <int T1, int T2>
struct MfmaShape {
  static constexpr int H1 = 32 * T1, H2 = 32 * T2;
  static constexpr int NP = H1 * kIn + H1 + H2 * H1 + H2 + 3 * H2 + 3;
  static constexpr int oW1 = 0, ob1 = H1 * kIn, oW2 = ob1 + H1, ob2 = oW2 + H2 * H1, oW3 = ob2 + H2,
                       ob3 = oW3 + 3 * H2;
  // LDS rows: x (16), h1, h2, dz1, dz2, dz3 (4: the last stays zero)
  static constexpr int rX = 0, rH1 = kIn, rH2 = rH1 + H1, rD1 = rH2 + H2, rD2 = rD1 + H1, rD3 = rD2 + H2,
                       rows = rD3 + 4;
  static constexpr int act_bytes = rows * kRow * 2;
  // the FP32 weights are staged in the same bytes before the rows are written
  static constexpr int lds_bytes = act_bytes > NP * 4 ? act_bytes : NP * 4;
};

template <int T1, int T2, bool FP8>
__global__ __launch_bounds__(64 * kMWaves) void train_mfma_kernel(TrainArgs a) {
  using S = MfmaShape<T1, T2>;
  constexpr int H1 = S::H1, H2 = S::H2, NP = S::NP;
  __shared__ __attribute__((aligned(16))) unsigned char smem[S::lds_bytes];
  __shared__ __attribute__((aligned(16))) float sB[H1 + H2 + 4];
  __shared__ float sLoss[kMWaves];
  __shared__ float sMax[3][kMWaves];
  float* sW = reinterpret_cast<float*>(smem);
  __bf16* sA = reinterpret_cast<__bf16*>(smem);
  auto row = [&](int r) { return sA + r * kRow; };
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, h = l >> 5, col = l & 31;

  for (int i = tid; i < NP; i += 64 * kMWaves) sW[i] = a.params[i];
  __syncthreads();
  // FP8: each layer's weight scale from the masters' largest magnitude, then
  // the weights in LDS replaced by their E4M3 values (the masters in HBM stay
  // FP32); activations use the caller's scales a.sa
  float sw0 = 1.0f, sw1 = 1.0f, sw2 = 1.0f;
  if constexpr (FP8) {
    float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f;
    for (int i = tid; i < H1 * kIn; i += 64 * kMWaves) m0 = fmaxf(m0, fabsf(sW[S::oW1 + i]));
    for (int i = tid; i < H2 * H1; i += 64 * kMWaves) m1 = fmaxf(m1, fabsf(sW[S::oW2 + i]));
    for (int i = tid; i < 3 * H2; i += 64 * kMWaves) m2 = fmaxf(m2, fabsf(sW[S::oW3 + i]));
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) {
      m0 = fmaxf(m0, __shfl_xor(m0, k));
      m1 = fmaxf(m1, __shfl_xor(m1, k));
      m2 = fmaxf(m2, __shfl_xor(m2, k));
    }
    if (l == 0) {
      sMax[0][wave] = m0;
      sMax[1][wave] = m1;
      sMax[2][wave] = m2;
    }
    __syncthreads();
    m0 = m1 = m2 = 0.0f;
#pragma unroll
    for (int w8 = 0; w8 < kMWaves; ++w8) {
      m0 = fmaxf(m0, sMax[0][w8]);
      m1 = fmaxf(m1, sMax[1][w8]);
      m2 = fmaxf(m2, sMax[2][w8]);
    }
    sw0 = e4m3_scale_for(m0);
    sw1 = e4m3_scale_for(m1);
    sw2 = e4m3_scale_for(m2);
    for (int i = tid; i < H1 * kIn; i += 64 * kMWaves) sW[S::oW1 + i] = fwd_value<true>(sW[S::oW1 + i], sw0, 1.0f / sw0);
    for (int i = tid; i < H2 * H1; i += 64 * kMWaves) sW[S::oW2 + i] = fwd_value<true>(sW[S::oW2 + i], sw1, 1.0f / sw1);
    for (int i = tid; i < 3 * H2; i += 64 * kMWaves) sW[S::oW3 + i] = fwd_value<true>(sW[S::oW3 + i], sw2, 1.0f / sw2);
    __syncthreads();
  }
  const float iw0 = 1.0f / sw0, iw1 = 1.0f / sw1, iw2 = 1.0f / sw2;  // exact: powers of two
  const float sa0 = FP8 ? a.sa[0] : 1.0f, sa1 = FP8 ? a.sa[1] : 1.0f, sa2 = FP8 ? a.sa[2] : 1.0f;
  const float ia0 = 1.0f / sa0, ia1 = 1.0f / sa1, ia2 = 1.0f / sa2;
  const float dq0 = sa0 * sw0, dq1 = sa1 * sw1, dq2 = sa2 * sw2;  // dequantisation of each layer's sums
  for (int i = tid; i < H1; i += 64 * kMWaves) sB[i] = sW[S::ob1 + i];
  for (int i = tid; i < H2; i += 64 * kMWaves) sB[H1 + i] = sW[S::ob2 + i];
  if (tid < 3) sB[H1 + H2 + tid] = sW[S::ob3 + tid];

  // ---- operands of the weights (every wave holds them) ----
  FwdVec<FP8> A1[T1], A2[T2][2 * T1], A3[2 * T2];
  bf16x8 A3T[T2], A2T[T1][2 * T2];
  float w[8];
#pragma unroll
  for (int t = 0; t < T1; ++t) {
    const int u = 32 * t + perm_row(col);
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = sW[S::oW1 + u * kIn + 8 * h + e];
    A1[t] = pack_fwd<FP8>(w, iw0);
  }
#pragma unroll
  for (int t = 0; t < T2; ++t) {
    const int u = 32 * t + perm_row(col);
#pragma unroll
    for (int c = 0; c < 2 * T1; ++c) {
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = sW[S::oW2 + u * H1 + 16 * c + 8 * h + e];
      A2[t][c] = pack_fwd<FP8>(w, iw1);
    }
    // W3^T: row = layer-2 unit u, K = output 8 h + e (three live)
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = (h == 0 && e < 3) ? sW[S::oW3 + e * H2 + u] : 0.0f;
    A3T[t] = pack8(w);
  }
#pragma unroll
  for (int c = 0; c < 2 * T2; ++c) {
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = col < 3 ? sW[S::oW3 + col * H2 + 16 * c + 8 * h + e] : 0.0f;
    A3[c] = pack_fwd<FP8>(w, iw2);
  }
  // W2^T: row = layer-1 unit j (permuted as layer 1), K = layer-2 unit 16 c + 8 h + e
#pragma unroll
  for (int t = 0; t < T1; ++t) {
    const int j = 32 * t + perm_row(col);
#pragma unroll
    for (int c = 0; c < 2 * T2; ++c) {
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = sW[S::oW2 + (16 * c + 8 * h + e) * H1 + j];
      A2T[t][c] = pack8(w);
    }
  }
  __syncthreads();  // the weight bytes become activation rows from here on
  for (int i = tid; i < kRow; i += 64 * kMWaves) row(S::rD3 + 3)[i] = static_cast<__bf16>(0.0f);

  // ---- this wave's 64 samples ----
  const int c0 = 64 * wave;                          // first column of the wave
  const int smp = blockIdx.x * kMSamples + c0 + l;   // this lane's sample
  const bool valid = smp < a.batch;
  float x[kIn];
#pragma unroll
  for (int c = 0; c < kIn; c += 4) {
    const float4 v = valid ? *reinterpret_cast<const float4*>(a.x + (size_t)smp * kIn + c)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
    x[c] = fwd_value<FP8>(v.x, sa0, ia0);
    x[c + 1] = fwd_value<FP8>(v.y, sa0, ia0);
    x[c + 2] = fwd_value<FP8>(v.z, sa0, ia0);
    x[c + 3] = fwd_value<FP8>(v.w, sa0, ia0);
  }
  float y[3];
#pragma unroll
  for (int o = 0; o < 3; ++o) y[o] = valid ? a.y[(size_t)smp * 3 + o] : 0.0f;
  const float wsmp = (valid && a.wt) ? a.wt[smp] : 1.0f;
#pragma unroll
  for (int c = 0; c < kIn; ++c) row(S::rX + c)[c0 + l] = static_cast<__bf16>(x[c]);
  // B operands of the two groups: half 0 takes inputs 0..7 and half 1
  // inputs 8..15 of sample `col` of the group
  float xa[8], xb[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float lo = x[e], hi = x[8 + e];
    const float lo_x = __shfl_xor(lo, 32), hi_x = __shfl_xor(hi, 32);
    xa[e] = h == 0 ? lo : hi_x;
    xb[e] = h == 0 ? lo_x : hi;
  }
  float lsum = 0.0f;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const FwdVec<FP8> XB = pack_fwd<FP8>(g == 0 ? xa : xb, ia0);
    const int sl = 32 * g + col;   // the wave's sample this lane's column stands for
    const int sc = c0 + sl;        // its LDS column
    // ---- layer 1 ----
    FwdVec<FP8> H1c[2 * T1];
    uint32_t m1[T1];
#pragma unroll
    for (int t = 0; t < T1; ++t) {
      f32x16 acc = {};
      acc = mfma_fwd<FP8>(A1[t], XB, acc);
      uint32_t m = 0;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float z = fmaf(acc[8 * c + e], dq0, sB[32 * t + 16 * c + 8 * h + e]);
          m |= (z > 0.0f ? 1u : 0u) << (8 * c + e);
          hv[e] = fwd_value<FP8>(fmaxf(z, 0.0f), sa1, ia1);
        }
        H1c[2 * t + c] = pack_fwd<FP8>(hv, ia1);
#pragma unroll
        for (int e = 0; e < 8; ++e) row(S::rH1 + 32 * t + 16 * c + 8 * h + e)[sc] = static_cast<__bf16>(hv[e]);
      }
      m1[t] = m;
    }
    // ---- layer 2 ----
    FwdVec<FP8> H2c[2 * T2];
    uint32_t m2[T2];
#pragma unroll
    for (int t = 0; t < T2; ++t) {
      f32x16 acc = {};
#pragma unroll
      for (int c = 0; c < 2 * T1; ++c) acc = mfma_fwd<FP8>(A2[t][c], H1c[c], acc);
      uint32_t m = 0;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float z = fmaf(acc[8 * c + e], dq1, sB[H1 + 32 * t + 16 * c + 8 * h + e]);
          m |= (z > 0.0f ? 1u : 0u) << (8 * c + e);
          hv[e] = fwd_value<FP8>(fmaxf(z, 0.0f), sa2, ia2);
        }
        H2c[2 * t + c] = pack_fwd<FP8>(hv, ia2);
#pragma unroll
        for (int e = 0; e < 8; ++e) row(S::rH2 + 32 * t + 16 * c + 8 * h + e)[sc] = static_cast<__bf16>(hv[e]);
      }
      m2[t] = m;
    }
    // ---- output, loss and dL/dz3 (half 0 holds the three outputs) ----
    f32x16 acc3 = {};
#pragma unroll
    for (int c = 0; c < 2 * T2; ++c) acc3 = mfma_fwd<FP8>(A3[c], H2c[c], acc3);
    const float yg0 = __shfl(y[0], sl), yg1 = __shfl(y[1], sl), yg2 = __shfl(y[2], sl);
    const float wg = __shfl(wsmp, sl);
    const bool vg = blockIdx.x * kMSamples + sc < a.batch;
    float d3[3] = {0.0f, 0.0f, 0.0f};
    if (h == 0 && vg) {
      const float yy[3] = {yg0, yg1, yg2};
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        const float z = fmaf(acc3[o], dq2, sB[H1 + H2 + o]);
        const float f = a.out_act ? 1.0f / (1.0f + expf(-z)) : fmaxf(z, 0.0f);
        const float e = f - yy[o];
        lsum = fmaf(wg * e * e, a.inv_count, lsum);
        const float df = a.out_act ? f * (1.0f - f) : (z > 0.0f ? 1.0f : 0.0f);
        d3[o] = q<true>(2.0f * wg * e * a.inv_count * df);
      }
    }
    if (h == 0) {
#pragma unroll
      for (int o = 0; o < 3; ++o) row(S::rD3 + o)[sc] = static_cast<__bf16>(d3[o]);
    }
    float dv[8] = {d3[0], d3[1], d3[2], 0.f, 0.f, 0.f, 0.f, 0.f};
    const bf16x8 D3B = pack8(dv);  // half 1 is all zero (d3 stays 0 there)
    // ---- dL/dz2 = (W3^T dz3) masked by layer 2's ReLU ----
    bf16x8 D2c[2 * T2];
#pragma unroll
    for (int t = 0; t < T2; ++t) {
      f32x16 acc = {};
      acc = mfma_bf16(A3T[t], D3B, acc);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float gv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) gv[e] = ((m2[t] >> (8 * c + e)) & 1u) ? acc[8 * c + e] : 0.0f;
        D2c[2 * t + c] = pack8(gv);
#pragma unroll
        for (int e = 0; e < 8; ++e) row(S::rD2 + 32 * t + 16 * c + 8 * h + e)[sc] = D2c[2 * t + c][e];
      }
    }
    // ---- dL/dz1 = (W2^T dz2) masked by layer 1's ReLU ----
#pragma unroll
    for (int t = 0; t < T1; ++t) {
      f32x16 acc = {};
#pragma unroll
      for (int c = 0; c < 2 * T2; ++c) acc = mfma_bf16(A2T[t][c], D2c[c], acc);
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float gv = ((m1[t] >> (8 * c + e)) & 1u) ? acc[8 * c + e] : 0.0f;
          row(S::rD1 + 32 * t + 16 * c + 8 * h + e)[sc] = static_cast<__bf16>(gv);
        }
    }
  }
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) lsum += __shfl_xor(lsum, k);
  if (l == 0) sLoss[wave] = lsum;
  __syncthreads();

  // ---- the block's gradient: K = its 256 samples ----
  float* out = a.partial + (size_t)blockIdx.x * NP;
  constexpr int kTiles = T2 * T1 + T1 + T2;
  const bf16x8 zero8 = {};
  for (int tile = wave; tile < kTiles; tile += kMWaves) {
    // which product: dW2 (t2, t1), dW1 (t1) or dW3 (t2); A rows / B columns
    const __bf16* arow;
    const __bf16* brow;
    bool alive, blive;
    if (tile < T2 * T1) {
      const int t2 = tile / T1, t1 = tile % T1;
      arow = row(S::rD2 + 32 * t2 + col); alive = true;
      brow = row(S::rH1 + 32 * t1 + col); blive = true;
    } else if (tile < T2 * T1 + T1) {
      const int t1 = tile - T2 * T1;
      arow = row(S::rD1 + 32 * t1 + col); alive = true;
      brow = row(S::rX + min(col, kIn - 1)); blive = col < kIn;
    } else {
      const int t2 = tile - T2 * T1 - T1;
      arow = row(S::rD3 + min(col, 3)); alive = col < 4;
      brow = row(S::rH2 + 32 * t2 + col); blive = true;
    }
    // two accumulators over alternating K steps, added at the end
    f32x16 acc0 = {}, acc1 = {};
#pragma unroll
    for (int ks = 0; ks < kMSamples / 16; ks += 2) {
      acc0 = mfma_bf16(alive ? lds8(arow + 16 * ks + 8 * h) : zero8, blive ? lds8(brow + 16 * ks + 8 * h) : zero8,
                       acc0);
      acc1 = mfma_bf16(alive ? lds8(arow + 16 * ks + 16 + 8 * h) : zero8,
                       blive ? lds8(brow + 16 * ks + 16 + 8 * h) : zero8, acc1);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float gsum = acc0[v] + acc1[v];
      const int r = 8 * (v >> 2) + 4 * h + (v & 3);  // accumulator row of register v
      if (tile < T2 * T1) {
        const int t2 = tile / T1, t1 = tile % T1;
        out[S::oW2 + (32 * t2 + r) * H1 + 32 * t1 + col] = gsum;
      } else if (tile < T2 * T1 + T1) {
        const int t1 = tile - T2 * T1;
        if (col < kIn) out[S::oW1 + (32 * t1 + r) * kIn + col] = gsum;
      } else {
        const int t2 = tile - T2 * T1 - T1;
        if (r < 3) out[S::oW3 + r * H2 + 32 * t2 + col] = gsum;
      }
    }
  }
  // bias gradients: thread i sums one dz row over the block's samples in order
  {
    int r = -1, o = 0;
    if (tid < H1) { r = S::rD1 + tid; o = S::ob1 + tid; }
    else if (tid < H1 + H2) { r = S::rD2 + tid - H1; o = S::ob2 + tid - H1; }
    else if (tid < H1 + H2 + 3) { r = S::rD3 + tid - H1 - H2; o = S::ob3 + tid - H1 - H2; }
    if (r >= 0) {
      float sum = 0.0f;
      for (int k = 0; k < kMSamples; k += 8) {
        const bf16x8 v = lds8(row(r) + k);
#pragma unroll
        for (int e = 0; e < 8; ++e) sum += static_cast<float>(v[e]);
      }
      out[o] = sum;
    }
  }
  if (tid == 0) a.partial_loss[blockIdx.x] = ((sLoss[0] + sLoss[1]) + sLoss[2]) + sLoss[3];
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

template <bool BF, int H1, int H2>
void launch_fb(const TrainArgs& t, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((train_fwd_bwd<BF, H1, H2>), dim3(nblocks), dim3(256), 0, s, t);
}

}  // namespace

size_t train_ws_bytes(int64_t batch, int64_t h1, int64_t h2) {
  if (batch <= 0 || h1 <= 0 || h2 <= 0) return 0;
  const int64_t nb = (batch + kSB - 1) / kSB;
  const int64_t np = h1 * kIn + h1 + h2 * h1 + h2 + 3 * h2 + 3;
  return align256((size_t)(nb * np) * 4) + align256((size_t)nb * 4);
}

int launch_train(const starnt_train& tr, const float* x, const float* y, int batch, const starnt_adam& hp,
                 float* loss, void* ws, size_t ws_bytes, hipStream_t s) {
  const int nb = (batch + kSB - 1) / kSB;
  const int np = tr.h1 * kIn + tr.h1 + tr.h2 * tr.h1 + tr.h2 + 3 * tr.h2 + 3;
  TrainArgs t;
  t.batch = batch;
  t.h1 = tr.h1;
  t.h2 = tr.h2;
  t.params = tr.params;
  t.x = x;
  t.y = y;
  t.wt = tr.weight;
  t.partial = static_cast<float*>(ws);
  t.partial_loss = reinterpret_cast<float*>(static_cast<char*>(ws) + align256((size_t)nb * np * 4));
  t.nparam = np;
  t.inv_count = (float)(1.0 / (3.0 * (double)batch));
  t.out_act = tr.out_act;
  const bool bf = tr.dtype == STARNT_BF16;
  bool ok = true;
  int nblocks = nb;
  // BF16 with hidden widths 32 or 64: the matrix-core kernel, kMSamples
  // samples per block
  const bool f8 = tr.dtype == STARNT_FP8;
  const bool mf = (bf || f8) && (tr.h1 == 32 || tr.h1 == 64) && (tr.h2 == 32 || tr.h2 == 64);
  if (f8 && !mf) return fail(STARNT_EUNSUPPORTED, "starnt_train_step: FP8 needs hidden widths of 32 or 64");
  for (int l = 0; l < 3; ++l) t.sa[l] = tr.fp8_act_scale[l];
  if (mf) {
    nblocks = (batch + kMSamples - 1) / kMSamples;
    const dim3 grid((unsigned)nblocks), block(64 * kMWaves);
    if (f8) {
      if (tr.h1 == 32 && tr.h2 == 32) hipLaunchKernelGGL((train_mfma_kernel<1, 1, true>), grid, block, 0, s, t);
      else if (tr.h1 == 32) hipLaunchKernelGGL((train_mfma_kernel<1, 2, true>), grid, block, 0, s, t);
      else if (tr.h2 == 32) hipLaunchKernelGGL((train_mfma_kernel<2, 1, true>), grid, block, 0, s, t);
      else hipLaunchKernelGGL((train_mfma_kernel<2, 2, true>), grid, block, 0, s, t);
    } else {
      if (tr.h1 == 32 && tr.h2 == 32) hipLaunchKernelGGL((train_mfma_kernel<1, 1, false>), grid, block, 0, s, t);
      else if (tr.h1 == 32) hipLaunchKernelGGL((train_mfma_kernel<1, 2, false>), grid, block, 0, s, t);
      else if (tr.h2 == 32) hipLaunchKernelGGL((train_mfma_kernel<2, 1, false>), grid, block, 0, s, t);
      else hipLaunchKernelGGL((train_mfma_kernel<2, 2, false>), grid, block, 0, s, t);
    }
  }
#define TCASE(A, B)                                                        \
  else if (tr.h1 == A && tr.h2 == B) {                                     \
    if (bf) launch_fb<true, A, B>(t, nb, s); else launch_fb<false, A, B>(t, nb, s); \
  }
  if (mf) {}
  TCASE(16, 16) TCASE(32, 16) TCASE(16, 32) TCASE(32, 32) TCASE(64, 64) TCASE(32, 64) TCASE(64, 32)
  else ok = false;
#undef TCASE
  if (!ok) return fail(STARNT_EUNSUPPORTED, "starnt_train_step: unsupported hidden widths");
  STARNT_LAUNCH_CHECK("starnt_train_step forward/backward launch");
  AdamArgs ad;
  ad.nparam = np;
  ad.nblocks = nblocks;
  ad.partial = t.partial;
  ad.partial_loss = t.partial_loss;
  ad.params = tr.params;
  ad.m = tr.m;
  ad.v = tr.v;
  ad.grad = tr.grad;
  ad.loss = loss;
  ad.lr = hp.lr;
  ad.b1 = hp.beta1;
  ad.b2 = hp.beta2;
  ad.eps = hp.eps;
  ad.c1 = (float)(1.0 - std::pow((double)hp.beta1, hp.step));
  ad.c2 = (float)(1.0 - std::pow((double)hp.beta2, hp.step));
  hipLaunchKernelGGL(train_reduce_adam, dim3((np + kRP - 1) / kRP), dim3(kRP * kRG), 0, s, ad);
  STARNT_LAUNCH_CHECK("starnt_train_step adam launch");
  (void)ws_bytes;
  return STARNT_OK;
}

}  // namespace starnt
