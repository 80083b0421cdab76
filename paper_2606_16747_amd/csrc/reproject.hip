// Interpolated frames by depth reprojection (Sec. 3.3): a gather from the last
// real frame using its first-fragment depth at the same pixel and the matrix
// M = VP_prev VP_cur^-1, given as M - I so the source offset is computed from
// the (small) motion, not from the absolute coordinates. A source outside the
// frame is clamped to the nearest edge pixel (reported as src = -1).
#include "internal.h"

namespace starnt {
namespace {

struct Mat4 {
  float m[16];
};

struct ReprojArgs {
  int W, H;
  const float* rgb;
  const float* d1;
  Mat4 d;  // M - I, row-major
  float* out;
  int32_t* src;
};

__global__ __launch_bounds__(256) void reproject_kernel(ReprojArgs a) {
  const int P = a.W * a.H;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int px, py;
  pixel_xy(p, a.W, px, py);
  const float X0 = (2.0f * px + 1.0f) / (float)a.W - 1.0f;
  const float X1 = 1.0f - (2.0f * py + 1.0f) / (float)a.H;
  const float X2 = a.d1[p];
  const float* d = a.d.m;
  // (M - I) X : the change of the homogeneous coordinates
  const float dx = fmaf(d[0], X0, fmaf(d[1], X1, fmaf(d[2], X2, d[3])));
  const float dy = fmaf(d[4], X0, fmaf(d[5], X1, fmaf(d[6], X2, d[7])));
  const float dw = fmaf(d[12], X0, fmaf(d[13], X1, fmaf(d[14], X2, d[15])));
  const float w = 1.0f + dw;
  int q = -1;
  int s = p;
  if (w > 0.0f) {
    // u - x = (dx - x dw) / w, in pixels: (u - x) W / 2; same for v (y up)
    const float ox = (dx - X0 * dw) / w * (0.5f * a.W);
    const float oy = (dy - X1 * dw) / w * (0.5f * a.H);
    // displacement in whole pixels, bounded so the integer conversion is safe
    const float fx = fminf(fmaxf(floorf(ox + 0.5f), -1e8f), 1e8f);
    const float fy = fminf(fmaxf(floorf(0.5f - oy), -1e8f), 1e8f);
    const long long qx = px + (long long)fx, qy = py + (long long)fy;
    if (qx >= 0 && qx < a.W && qy >= 0 && qy < a.H) q = (int)(qy * a.W + qx);
    // outside the frame: edge extension (src stays -1)
    const int cx = (int)(qx < 0 ? 0 : (qx > a.W - 1 ? a.W - 1 : qx));
    const int cy = (int)(qy < 0 ? 0 : (qy > a.H - 1 ? a.H - 1 : qy));
    s = cy * a.W + cx;
  }
  a.out[3 * (size_t)p + 0] = a.rgb[3 * (size_t)s + 0];
  a.out[3 * (size_t)p + 1] = a.rgb[3 * (size_t)s + 1];
  a.out[3 * (size_t)p + 2] = a.rgb[3 * (size_t)s + 2];
  if (a.src) a.src[p] = q;
}

}  // namespace

int launch_reproject(const float* rgb_prev, const float* d1_prev, int W, int H, const float mmi[16],
                     float* rgb_out, int32_t* src, hipStream_t s) {
  ReprojArgs a;
  a.W = W;
  a.H = H;
  a.rgb = rgb_prev;
  a.d1 = d1_prev;
  for (int i = 0; i < 16; ++i) a.d.m[i] = mmi[i];
  a.out = rgb_out;
  a.src = src;
  const int P = W * H;
  hipLaunchKernelGGL(reproject_kernel, dim3((P + 255) / 256), dim3(256), 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_reproject launch");
  return STARNT_OK;
}

}  // namespace starnt
