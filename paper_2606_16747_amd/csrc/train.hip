// Training step of the tail-colour network (Sec. 3.3: MSE loss, Adam), on the
// GPU with FP32 master weights.
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
  float* partial;       // [nblocks][nparam]
  float* partial_loss;  // [nblocks]
  int nparam;
  float inv_count;      // 1 / (batch * 3)
  int out_act;          // 0 ReLU, 1 logistic sigmoid
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
      lsum = fmaf(e * e, a.inv_count, lsum);
      const float df = a.out_act ? f * (1.0f - f) : (z > 0.0f ? 1.0f : 0.0f);
      d = 2.0f * e * a.inv_count * df;
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
  if (i < a.nparam)
    for (int b = r; b < a.nblocks; b += kRG) g += a.partial[(size_t)b * a.nparam + i];
  s_part[r][c] = g;
  __syncthreads();
  if (r == 0 && i < a.nparam) {
    float t = 0.0f;
    for (int k = 0; k < kRG; ++k) t += s_part[k][c];
    a.grad[i] = t;
    const float m = fmaf(a.b1, a.m[i], (1.0f - a.b1) * t);
    const float v = fmaf(a.b2, a.v[i], (1.0f - a.b2) * t * t);
    a.m[i] = m;
    a.v[i] = v;
    const float mh = m / a.c1, vh = v / a.c2;
    a.params[i] -= a.lr * mh / (sqrtf(vh) + a.eps);
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
  t.partial = static_cast<float*>(ws);
  t.partial_loss = reinterpret_cast<float*>(static_cast<char*>(ws) + align256((size_t)nb * np * 4));
  t.nparam = np;
  t.inv_count = (float)(1.0 / (3.0 * (double)batch));
  t.out_act = tr.out_act;
  const bool bf = tr.dtype == STARNT_BF16;
  bool ok = true;
#define TCASE(A, B)                                                        \
  else if (tr.h1 == A && tr.h2 == B) {                                     \
    if (bf) launch_fb<true, A, B>(t, nb, s); else launch_fb<false, A, B>(t, nb, s); \
  }
  if (false) {}
  TCASE(16, 16) TCASE(32, 16) TCASE(16, 32) TCASE(32, 32) TCASE(64, 64) TCASE(32, 64) TCASE(64, 32)
  else ok = false;
#undef TCASE
  if (!ok) return fail(STARNT_EUNSUPPORTED, "starnt_train_step: unsupported hidden widths");
  STARNT_LAUNCH_CHECK("starnt_train_step forward/backward launch");
  AdamArgs ad;
  ad.nparam = np;
  ad.nblocks = nb;
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
