// Interpolated frames by depth reprojection (Sec. 3.3): a gather from the last
// real frame using its first-fragment depth at the same pixel and the matrix
// M = VP_prev VP_cur^-1, given as M - I so the source offset is computed from
// the (small) motion, not from the absolute coordinates. A source outside the
// frame is clamped to the nearest edge pixel (reported as src = -1).
//
// With a depth tolerance the gather also says which pixels it cannot trust:
// besides the pixels whose source is outside the frame or behind the camera,
// those whose source pixel's first-fragment depth differs from the
// reprojected depth z' = h_z / h_w by more than the tolerance (the source
// shows another surface: a disocclusion or a depth edge), src = -2. Untrusted
// pixels are appended to a list for re-rendering; a wave takes its slots with
// one atomic, so the list's order varies between runs, its contents do not.
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
  float tol;          // depth tolerance, 0: no depth test
  uint32_t* list;     // untrusted pixels (optional)
  uint32_t* list_n;   // their number, zero on entry
};

__global__ void clear_count_kernel(uint32_t* n) { *n = 0u; }

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
  const float dz = fmaf(d[8], X0, fmaf(d[9], X1, fmaf(d[10], X2, d[11])));
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
    if (qx >= 0 && qx < a.W && qy >= 0 && qy < a.H) {
      q = (int)(qy * a.W + qx);
      // reprojected depth against the depth the source pixel holds
      if (a.tol > 0.0f && fabsf(a.d1[q] - (X2 + dz) / w) > a.tol) q = -2;
    }
    // outside the frame: edge extension (src stays -1)
    const int cx = (int)(qx < 0 ? 0 : (qx > a.W - 1 ? a.W - 1 : qx));
    const int cy = (int)(qy < 0 ? 0 : (qy > a.H - 1 ? a.H - 1 : qy));
    s = cy * a.W + cx;
  }
  a.out[3 * (size_t)p + 0] = a.rgb[3 * (size_t)s + 0];
  a.out[3 * (size_t)p + 1] = a.rgb[3 * (size_t)s + 1];
  a.out[3 * (size_t)p + 2] = a.rgb[3 * (size_t)s + 2];
  if (a.src) a.src[p] = q;
  if (a.list) {
    const bool bad = q < 0;
    const uint64_t m = __builtin_amdgcn_ballot_w64(bad);
    if (m != 0) {
      const int lane = (int)__lane_id();
      const int leader = __builtin_ctzll(m);
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(a.list_n, (uint32_t)__builtin_popcountll(m));
      base = __shfl(base, leader);
      if (bad) a.list[base + (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull))] = (uint32_t)p;
    }
  }
}

}  // namespace

int launch_reproject(const float* rgb_prev, const float* d1_prev, int W, int H, const float mmi[16],
                     float* rgb_out, int32_t* src, hipStream_t s, float tol, uint32_t* list, uint32_t* list_n) {
  ReprojArgs a;
  a.W = W;
  a.H = H;
  a.rgb = rgb_prev;
  a.d1 = d1_prev;
  for (int i = 0; i < 16; ++i) a.d.m[i] = mmi[i];
  a.out = rgb_out;
  a.src = src;
  a.tol = tol;
  a.list = list;
  a.list_n = list_n;
  const int P = W * H;
  // a fill kernel rather than a memset, so a captured graph replays it safely
  if (list) hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(1), 0, s, list_n);
  hipLaunchKernelGGL(reproject_kernel, dim3((P + 255) / 256), dim3(256), 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_reproject launch");
  return STARNT_OK;
}

}  // namespace starnt
