// Internal declarations of libstarnt: launch helpers shared by the kernels and
// the C-ABI layer. Device helpers here are used by GPU code only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/starnt.h"

namespace starnt {

// ---- error reporting (thread-local message, status code) -----------------
int fail(int code, const std::string& msg);
int hip_status(hipError_t e, const char* what);

#define STARNT_LAUNCH_CHECK(what)                         \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return hip_status(e_, what);    \
  } while (0)

// ---- device helpers -------------------------------------------------------

// Grid index i of the W_s-sample grid that samples full-resolution coordinate
// x (sample i sits at floor((2i+1) W / (2 W_s))), or -1 when x is not sampled.
__device__ __forceinline__ int grid_index_of(int x, int W, int Ws) {
  if (Ws >= W) return x;
  // smallest i with (2i+1) W >= 2 Ws x
  long long num = 2LL * Ws * x - W;
  long long den = 2LL * W;
  long long i = num <= 0 ? 0 : (num + den - 1) / den;
  if (i >= Ws) return -1;
  long long pos = ((2 * i + 1) * (long long)W) / (2LL * Ws);
  return pos == x ? (int)i : -1;
}

// Bilinear taps along one axis for full-resolution coordinate x on a W_s grid:
// grid coordinate u = ((2x+1) W_s - W) / (2W), taps floor(u) and floor(u)+1
// clamped to [0, W_s-1], weight of the upper tap = frac(u).
struct Taps {
  int i0, i1;
  float w1;
};
__device__ __forceinline__ Taps axis_taps(int x, int W, int Ws) {
  Taps t;
  long long num = (2LL * x + 1) * Ws - W;
  long long den = 2LL * W;
  long long q = num >= 0 ? num / den : -((-num + den - 1) / den);
  long long r = num - q * den;
  t.w1 = (float)r / (float)den;
  long long a = q < 0 ? 0 : (q > Ws - 1 ? Ws - 1 : q);
  long long b = q + 1 < 0 ? 0 : (q + 1 > Ws - 1 ? Ws - 1 : q + 1);
  t.i0 = (int)a;
  t.i1 = (int)b;
  return t;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// grid sizes from a device schedule (NULL = full resolution), clamped to the frame
struct Grids {
  int w2, h2, w3, h3;
};
__device__ __forceinline__ Grids load_grids(const starnt_sched* s, int W, int H) {
  Grids g;
  if (!s) {
    g.w2 = W; g.h2 = H; g.w3 = W; g.h3 = H;
    return g;
  }
  g.w2 = clampi(s->w2, 1, W);
  g.h2 = clampi(s->h2, 1, H);
  g.w3 = clampi(s->w3, 1, W);
  g.h3 = clampi(s->h3, 1, H);
  return g;
}

// RGBA fetch of fragment k (straight colour)
template <bool HALF>
__device__ __forceinline__ float4 load_rgba(const void* rgba, uint32_t k) {
  if constexpr (HALF) {
    typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
    const half4_t h = reinterpret_cast<const half4_t*>(rgba)[k];
    return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
  } else {
    return reinterpret_cast<const float4*>(rgba)[k];
  }
}

// ---- launchers (one per kernel family) -------------------------------------
int launch_features(const starnt_frags& f, const starnt_sched* sched, const starnt_feats& o, hipStream_t s);
int launch_exact(const starnt_frags& f, const float bg[3], float* rgb, float* fstar, uint32_t* err,
                 hipStream_t s);
int launch_composite(const starnt_feats& o, const float* tail_rgb, const starnt_sched* sched, int W, int H,
                     const float bg[3], int mode, float* rgb, hipStream_t s);
int launch_infer(const starnt_mlp& m, const float* tail, const uint32_t* count, const starnt_sched* sched,
                 int W, int H, float* out, hipStream_t s);
int launch_quadtree(const float* rgb, const uint32_t* count, int W, int H, const starnt_qt_params& qp,
                    const uint32_t* prev_mask, uint32_t* mask, uint8_t* level, starnt_sched* sched, void* ws,
                    hipStream_t s);
size_t quadtree_ws_bytes(int64_t W, int64_t H, int64_t base);
int launch_reproject(const float* rgb_prev, const float* d1_prev, int W, int H, const float mmi[16],
                     float* rgb_out, int32_t* src, hipStream_t s);
int launch_train(const starnt_train& t, const float* x, const float* y, int batch, const starnt_adam& hp,
                 float* loss, void* ws, size_t ws_bytes, hipStream_t s);
size_t train_ws_bytes(int64_t batch, int64_t h1, int64_t h2);
int launch_sched_init(starnt_sched* sched, int w2, int h2, int w3, int h3, hipStream_t s);

}  // namespace starnt
