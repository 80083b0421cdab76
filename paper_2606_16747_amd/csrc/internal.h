// Internal declarations of libstarnt: launch helpers shared by the kernels and
// the C-ABI layer. Device helpers here are used by GPU code only.
#pragma once

#include <hip/hip_ext.h>
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

// ---- kernel timing (starnt_time_next_launch) -------------------------------
// The pending request of the calling thread, taken (and cleared) by the
// launcher of the timed kernel.
struct LaunchTimer {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTimer take_launch_timer();

// hipLaunchKernelGGL, or hipExtLaunchKernelGGL recording the timer's events
// with the dispatch itself when a request is pending
template <typename K, typename... Args>
void launch_maybe_timed(const LaunchTimer& tm, K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
  if (tm.start || tm.stop) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, tm.start, tm.stop, 0, args...);
  else hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// ---- device helpers -------------------------------------------------------

// a * b for a, b < 2^24 with a product below 2^32, exactly: one full-rate
// v_mul_u32_u24 (a 32-bit v_mul_lo_u32 takes four issue cycles). Frame and
// grid sides are at most 16384, so every index product here qualifies.
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) { return __umul24(a, b); }

// floor(n / d) for n < 2^30, 1 <= d < 2^24 and a quotient below 2^15, exactly.
// The FP32 estimate n * rcp(d) carries a relative error below 2^-22 (n rounded
// once, the hardware reciprocal within 1 ulp, the product rounded once), so its
// absolute error is below 2^-7 and its truncation is the true quotient or one
// off; the remainder's sign and size fix that one step. About a third of the
// instructions of the general 32-bit division.
__device__ __forceinline__ uint32_t udiv_small(uint32_t n, uint32_t d) {
  const float f = (float)n * __builtin_amdgcn_rcpf((float)d);
  uint32_t q = (uint32_t)f;
  const int32_t r = (int32_t)(n - mul24(q, d));
  q = r < 0 ? q - 1u : (r >= (int32_t)d ? q + 1u : q);
  return q;
}

// Pixel coordinates of linear pixel index p in a frame of width W.
__device__ __forceinline__ void pixel_xy(int p, int W, int& x, int& y) {
  y = (int)udiv_small((uint32_t)p, (uint32_t)W);
  x = p - (int)mul24((uint32_t)y, (uint32_t)W);
}

// Grid index i of the W_s-sample grid that samples full-resolution coordinate
// x (sample i sits at floor((2i+1) W / (2 W_s))), or -1 when x is not sampled.
// The candidate is the smallest i with (2i+1) W >= 2 W_s x; it samples x iff
// (2i+1) W < 2 W_s (x+1) as well. Frame sides are at most 16384, so every
// product is below 2^30, every quotient at most 16384, and the 32-bit
// arithmetic is exact.
__device__ __forceinline__ int grid_index_of(int x, int W, int Ws) {
  if (Ws >= W) return x;
  const int num = (int)mul24(2u * Ws, (uint32_t)x) - W;
  const int den = 2 * W;
  const int i = num <= 0 ? 0 : (int)udiv_small((unsigned)num + (unsigned)den - 1u, (unsigned)den);
  return (i < Ws && mul24(2u * i + 1u, (uint32_t)W) < mul24(2u * Ws, (uint32_t)x + 1u)) ? i : -1;
}

// Bilinear taps along one axis for full-resolution coordinate x on a W_s grid:
// grid coordinate u = ((2x+1) W_s - W) / (2W), taps floor(u) and floor(u)+1
// clamped to [0, W_s-1], weight of the upper tap = frac(u) (the exact integer
// remainder times the hardware reciprocal of 2W, within 2 ulp).
struct Taps {
  int i0, i1;
  float w1;
};
__device__ __forceinline__ Taps axis_taps(int x, int W, int Ws) {
  Taps t;
  const int num = (int)mul24(2u * x + 1u, (uint32_t)Ws) - W;  // >= -W
  const int den = 2 * W;
  // floor division for num >= -den
  const int q = num >= 0 ? (int)udiv_small((unsigned)num, (unsigned)den) : -1;
  const int r = q < 0 ? num + den : num - (int)mul24((uint32_t)q, (uint32_t)den);
  t.w1 = (float)r * __builtin_amdgcn_rcpf((float)den);  // 0 exactly when r = 0
  t.i0 = q < 0 ? 0 : (q > Ws - 1 ? Ws - 1 : q);
  t.i1 = q + 1 < 0 ? 0 : (q + 1 > Ws - 1 ? Ws - 1 : q + 1);
  return t;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---- matrix-core operands (v_mfma_f32_32x32x16_bf16) ----------------------
// A: lane l holds row l % 32, K elements 8 (l / 32) .. + 7; B: lane l holds
// column l % 32, the same K elements; C/D: lane l holds column l % 32,
// register v is row 8 (v / 4) + 4 (l / 32) + v % 4.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// E4M3 operands of v_mfma_f32_32x32x16_fp8_fp8: the same lane layout as the
// bf16 operands above, 8 one-byte values per lane.
typedef long fp8x8;

// OCP E4M3 of four values, round-to-nearest-even (hardware convert); callers
// saturate to +-448 first
__device__ __forceinline__ uint32_t e4m3_pack4(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}
__device__ __forceinline__ float sat448(float v) { return fminf(fmaxf(v, -448.0f), 448.0f); }
// the E4M3 value nearest to v (saturated), as a float
__device__ __forceinline__ float e4m3_value(float v) {
  const int w = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v), 0.0f, 0, false);
  return __builtin_amdgcn_cvt_f32_fp8(w, 0);
}

// Physical accumulator row r of a 32-row tile (lane half h = (r % 8) / 4,
// block b = r / 8, element i = r % 4) holds logical hidden unit
// 16 (b / 2) + 8 h + 4 (b % 2) + i, so that accumulator register v = 4 b + i
// of lane half h is element (v % 8) of B-operand chunk (v / 8) for the next
// layer (chunk K index 8 h + e).
__device__ __forceinline__ int perm_row(int r) {
  const int b = r >> 3, h = (r >> 2) & 1, i = r & 3;
  return 16 * (b >> 1) + 8 * h + 4 * (b & 1) + i;
}

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
int launch_infer_composite_sel(const starnt_mlp& m, const starnt_feats& f, const starnt_sched* sched,
                               const uint8_t* level, int base, const float bg[3], float* rgb, hipStream_t s);
int launch_dfa_inputs(const starnt_feats& f, const starnt_sched* sched, float* x, hipStream_t s);
int launch_baseline(const starnt_frags& f, int32_t method, const float bg[3], float* rgb, hipStream_t s);
int launch_composite(const starnt_feats& o, const float* tail_rgb, const starnt_sched* sched, int W, int H,
                     const float bg[3], int mode, float* rgb, hipStream_t s);
int launch_infer(const starnt_mlp& m, const float* tail, const uint32_t* count, const starnt_sched* sched,
                 int W, int H, float* out, hipStream_t s);
int launch_infer_composite(const starnt_mlp& m, const starnt_feats& f, const starnt_sched* sched,
                           const float bg[3], float* rgb, hipStream_t s);
int launch_quadtree(const float* rgb, const uint32_t* count, int W, int H, const starnt_qt_params& qp,
                    const uint32_t* prev_mask, uint32_t* mask, uint8_t* level, starnt_sched* sched, void* ws,
                    hipStream_t s);
size_t quadtree_ws_bytes(int64_t W, int64_t H, int64_t base);
int launch_quadtree_noalloc(const float* rgb, const uint32_t* count, int W, int H, const starnt_qt_params& qp,
                            const uint32_t* prev_mask, uint32_t* mask, uint8_t* level, starnt_sched* sched,
                            hipStream_t s);
size_t quadtree_scratch_bytes();
int launch_reproject(const float* rgb_prev, const float* d1_prev, int W, int H, const float mmi[16],
                     float* rgb_out, int32_t* src, hipStream_t s, float tol = 0.0f, uint32_t* list = nullptr,
                     uint32_t* list_n = nullptr, void* ws = nullptr);
size_t reproject_ws_bytes(int64_t W, int64_t H);
int launch_features_list(const starnt_frags& f, const uint32_t* list, const uint32_t* list_n,
                         const starnt_feats& slots, hipStream_t s);
int launch_infer_patch(const starnt_mlp& m, const starnt_feats& slots, const uint32_t* list,
                       const uint32_t* list_n, uint32_t frame_p, const float bg[3], float* rgb, hipStream_t s);
int launch_train(const starnt_train& t, const float* x, const float* y, int batch, const starnt_adam& hp,
                 float* loss, void* ws, size_t ws_bytes, hipStream_t s);
size_t train_ws_bytes(int64_t batch, int64_t h1, int64_t h2);
int launch_sched_init(starnt_sched* sched, int w2, int h2, int w3, int h3, hipStream_t s);

}  // namespace starnt
