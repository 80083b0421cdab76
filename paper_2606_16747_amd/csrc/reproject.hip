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
// pixels are compacted into a list in increasing pixel order for
// re-rendering, without atomics (thousands of waves appending to one counter
// serialise on it): the gather writes one ballot mask per wave and one count
// per block; a scatter kernel then writes each wave's pixels at its block's
// offset, the sum of the earlier blocks' counts, which every scatter block
// forms itself with one coalesced block-wide sum (no separate scan launch),
// plus the counts of the block's earlier waves.
#include "internal.h"

namespace starnt {
namespace {

constexpr int kBlock = 1024;              // pixels (threads) per block
constexpr int kWaves = kBlock / 64;       // waves per block

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
  uint64_t* mask;     // per wave: untrusted lanes (trust test only)
  uint32_t* bcount;   // per block: untrusted pixels (trust test only)
};

__device__ __forceinline__ uint32_t popc64(uint64_t v) { return (uint32_t)__builtin_popcountll(v); }

__global__ __launch_bounds__(kBlock) void reproject_kernel(ReprojArgs a) {
  const int P = a.W * a.H;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = p < P;
  int q = -1;
  if (valid) {
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
    // all three loads before any store: stores ahead of a load to memory that
    // might alias would each wait for the load (three round trips, not one);
    // the entry points reject an output that overlaps an input
    const float c0 = a.rgb[3 * (size_t)s + 0], c1 = a.rgb[3 * (size_t)s + 1], c2 = a.rgb[3 * (size_t)s + 2];
    a.out[3 * (size_t)p + 0] = c0;
    a.out[3 * (size_t)p + 1] = c1;
    a.out[3 * (size_t)p + 2] = c2;
    if (a.src) a.src[p] = q;
  }
  if (a.mask) {  // uniform over the launch
    __shared__ uint32_t s_cnt[kWaves];
    const uint64_t m = __builtin_amdgcn_ballot_w64(valid && q < 0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // lane 0 holds the wave's lowest pixel, so it is valid iff any lane is
    if (lane == 0) {
      if (valid) a.mask[p >> 6] = m;
      s_cnt[wave] = popc64(m);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t c = 0;
      for (int i = 0; i < kWaves; ++i) c += s_cnt[i];
      a.bcount[blockIdx.x] = c;
    }
  }
}

// each wave writes its untrusted pixels, in lane (pixel) order, at the
// block's offset plus the counts of the block's earlier waves; the last block
// also writes the list's length
__global__ __launch_bounds__(kBlock) void scatter_list_kernel(const uint64_t* mask, const uint32_t* bcount, int nb,
                                                               int P, uint32_t* list, uint32_t* total) {
  __shared__ uint32_t s_cnt[kWaves];
  __shared__ uint32_t s_part[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w = blockIdx.x * kWaves + wave;  // global wave index
  const int p = blockIdx.x * kBlock + threadIdx.x;
  const bool live = w * 64 < P;              // the wave covers a pixel
  const uint64_t m = live ? mask[w] : 0ull;
  // offset of this block: sum of the earlier blocks' counts
  uint32_t part = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kBlock) part += bcount[b];
  for (int k = 32; k >= 1; k >>= 1) part += __shfl_xor(part, k);
  if (lane == 0) {
    s_cnt[wave] = popc64(m);
    s_part[wave] = part;
  }
  __syncthreads();
  uint32_t base = 0;
  for (int i = 0; i < kWaves; ++i) base += s_part[i];
  for (int i = 0; i < wave; ++i) base += s_cnt[i];
  if ((m >> lane) & 1ull) list[base + popc64(m & ((1ull << lane) - 1ull))] = (uint32_t)p;
  if (blockIdx.x == nb - 1 && threadIdx.x == kBlock - 1) *total = base + s_cnt[kWaves - 1];
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

size_t reproject_ws_bytes(int64_t W, int64_t H) {
  if (W <= 0 || H <= 0) return 0;
  const int64_t P = W * H;
  const int64_t nb = (P + kBlock - 1) / kBlock;
  return align256((size_t)((P + 63) / 64) * 8) + align256((size_t)nb * 4);
}

int launch_reproject(const float* rgb_prev, const float* d1_prev, int W, int H, const float mmi[16],
                     float* rgb_out, int32_t* src, hipStream_t s, float tol, uint32_t* list, uint32_t* list_n,
                     void* ws) {
  ReprojArgs a;
  a.W = W;
  a.H = H;
  a.rgb = rgb_prev;
  a.d1 = d1_prev;
  for (int i = 0; i < 16; ++i) a.d.m[i] = mmi[i];
  a.out = rgb_out;
  a.src = src;
  a.tol = tol;
  const int P = W * H;
  const int nb = (P + kBlock - 1) / kBlock;
  if (list) {
    uint8_t* base = static_cast<uint8_t*>(ws);
    a.mask = reinterpret_cast<uint64_t*>(base);
    a.bcount = reinterpret_cast<uint32_t*>(base + align256((size_t)((P + 63) / 64) * 8));
  } else {
    a.mask = nullptr;
    a.bcount = nullptr;
  }
  hipLaunchKernelGGL(reproject_kernel, dim3(nb), dim3(kBlock), 0, s, a);
  if (list) hipLaunchKernelGGL(scatter_list_kernel, dim3(nb), dim3(kBlock), 0, s, a.mask, a.bcount, nb, P, list, list_n);
  STARNT_LAUNCH_CHECK("starnt_reproject launch");
  return STARNT_OK;
}

}  // namespace starnt
