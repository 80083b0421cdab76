// Decoupled composite of STAR-NT (eq (3), Sec. 3.3) at full resolution:
//   C = a1 c1 + (1 - a1) a2 c2 + T2 f + T2 t_tail C_b,  T2 = (1 - a1)(1 - a2),
// with layer 1 from pass 1 (full resolution) and (a2, a2 c2), t_tail and the
// network input upscaled bilinearly from the pass-2 / pass-3 grids (Sec. 3.2).
// The full-resolution count N gates the upscaled terms: no second layer where
// N < 2, no tail where N < 3.
#include "internal.h"

namespace starnt {
namespace {

struct CompArgs {
  int W, H;
  const float4* layer1;
  const uint32_t* count;
  const float4* layer2;
  const float4* tail;
  const float* tail_rgb;
  const starnt_sched* sched;
  int mode;
  float bg0, bg1, bg2;
  float* rgb;
};

__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float w) {
  return make_float4(fmaf(w, b.x - a.x, a.x), fmaf(w, b.y - a.y, a.y), fmaf(w, b.z - a.z, a.z),
                     fmaf(w, b.w - a.w, a.w));
}

// bilinear fetch of a float4 field stored with `stride` float4 per sample
__device__ __forceinline__ float4 bilerp(const float4* g, int stride, int comp, int Ws, Taps tx, Taps ty) {
  const float4 v00 = g[((size_t)ty.i0 * Ws + tx.i0) * stride + comp];
  const float4 v01 = g[((size_t)ty.i0 * Ws + tx.i1) * stride + comp];
  const float4 v10 = g[((size_t)ty.i1 * Ws + tx.i0) * stride + comp];
  const float4 v11 = g[((size_t)ty.i1 * Ws + tx.i1) * stride + comp];
  return lerp4(lerp4(v00, v01, tx.w1), lerp4(v10, v11, tx.w1), ty.w1);
}

__global__ __launch_bounds__(256) void composite_kernel(CompArgs a) {
  const int P = a.W * a.H;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const Grids g = load_grids(a.sched, a.W, a.H);
  int x, y;
  pixel_xy(p, a.W, x, y);
  const uint32_t n = a.count[p];
  const float4 l1 = a.layer1[p];
  float4 l2 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (n >= 2) {
    const Taps tx = axis_taps(x, a.W, g.w2), ty = axis_taps(y, a.H, g.h2);
    l2 = bilerp(a.layer2, 1, 0, g.w2, tx, ty);
  }
  float f0 = 0.f, f1 = 0.f, f2 = 0.f, tt = 1.0f;
  if (n >= 3) {
    const Taps tx = axis_taps(x, a.W, g.w3), ty = axis_taps(y, a.H, g.h3);
    const float4 t0 = bilerp(a.tail, 2, 0, g.w3, tx, ty);  // N, t_tail, Ct_r, Ct_g
    tt = t0.y;
    if (a.mode == STARNT_MODE_LEARNED) {
      f0 = a.tail_rgb[3 * (size_t)p + 0];
      f1 = a.tail_rgb[3 * (size_t)p + 1];
      f2 = a.tail_rgb[3 * (size_t)p + 2];
    } else if (a.mode == STARNT_MODE_FAVG) {
      const float4 t1 = bilerp(a.tail, 2, 1, g.w3, tx, ty);  // Ct_b, ...
      const float w = 1.0f - tt;
      f0 = t0.z * w;
      f1 = t0.w * w;
      f2 = t1.x * w;
    }
  }
  const float a1 = l1.w, a2 = l2.w;
  const float om1 = 1.0f - a1;
  const float T2 = om1 * (1.0f - a2);
  const float Tb = T2 * tt;
  a.rgb[3 * (size_t)p + 0] = l1.x + om1 * l2.x + T2 * f0 + Tb * a.bg0;
  a.rgb[3 * (size_t)p + 1] = l1.y + om1 * l2.y + T2 * f1 + Tb * a.bg1;
  a.rgb[3 * (size_t)p + 2] = l1.z + om1 * l2.z + T2 * f2 + Tb * a.bg2;
}

}  // namespace

int launch_composite(const starnt_feats& o, const float* tail_rgb, const starnt_sched* sched, int W, int H,
                     const float bg[3], int mode, float* rgb, hipStream_t s) {
  CompArgs a;
  a.W = W;
  a.H = H;
  a.layer1 = reinterpret_cast<const float4*>(o.layer1);
  a.count = o.count;
  a.layer2 = reinterpret_cast<const float4*>(o.layer2);
  a.tail = reinterpret_cast<const float4*>(o.tail);
  a.tail_rgb = tail_rgb;
  a.sched = sched;
  a.mode = mode;
  a.bg0 = bg[0];
  a.bg1 = bg[1];
  a.bg2 = bg[2];
  a.rgb = rgb;
  const int P = W * H;
  hipLaunchKernelGGL(composite_kernel, dim3((P + 255) / 256), dim3(256), 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_composite launch");
  return STARNT_OK;
}

}  // namespace starnt
