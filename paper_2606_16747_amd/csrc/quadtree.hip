// Screen-tile quadtree of STAR-NT (Sec. 3.1) and the pass scales it implies
// for the next frame (Sec. 3.2, eq (4)).
//
// A base tile of B px is a 4-level quadtree: nodes of B, B/2, B/4 px can split;
// the B/8-px cells are leaves. Split state lives in a 21-bit mask per tile
// (bit 0 root, 1-4 level 1, 5-20 level 2, Morton order).
//
// One 64-lane wave per tile, one lane per cell:
//  pass 0 (top-down): the 8 x 8 unique corner samples of the tile's 21 internal
//    nodes are staged in LDS; D of each node = mean pairwise RGB distance of its
//    4 corners; split/merge with hysteresis top-down; per-cell leaf level,
//    limited to +-1 from the previous mask; masks re-derived from the levels.
//  pass 1..k (relaxation, global): r(c) = max(L(c), max over 4-neighbours - 1),
//    masks re-derived (node at level l split iff a cell under it has r > l,
//    via wave ballots), leaf levels re-read.
//  The last pass writes masks, levels and per-tile occupied-leaf counts; a
//  one-block kernel sums them in a fixed order and computes wbar, s2, s3 and
//  the next grids on the device.
#include "internal.h"

namespace starnt {
namespace {

struct QtArgs {
  int W, H, B, Tw, Th, Cw, Ch;
  float tau_split, tau_merge;
  const float* rgb;
  const uint32_t* count;
  const uint32_t* prev_mask;
  const uint8_t* Lin;
  uint8_t* Lout;
  uint32_t* mask;
  uint8_t* level;
  uint32_t* tile_hist;  // [T][4]
  int mode;             // 0 top-down, 1 relaxation
  int final_pass;
};

__device__ __forceinline__ int leaf_of(uint32_t m, int cx, int cy) {
  if (!(m & 1u)) return 0;
  const int q = (cx >> 2) + 2 * (cy >> 2);
  if (!(m & (1u << (1 + q)))) return 1;
  const int n2 = 5 + 4 * q + ((cx >> 1) & 1) + 2 * ((cy >> 1) & 1);
  if (!(m & (1u << n2))) return 2;
  return 3;
}

__device__ __forceinline__ int bit_of(int lvl, int nx, int ny) {
  if (lvl == 0) return 0;
  if (lvl == 1) return 1 + nx + 2 * ny;
  return 5 + 4 * ((nx >> 1) + 2 * (ny >> 1)) + (nx & 1) + 2 * (ny & 1);
}

__device__ __forceinline__ uint64_t node_cells(int lvl, int nx, int ny) {
  if (lvl == 0) return ~0ull;
  if (lvl == 1) return 0x0F0F0F0Full << (4 * nx + 32 * ny);
  return 0x0303ull << (2 * nx + 16 * ny);
}

// mask from per-cell levels (lane = cell, live = cell inside the frame)
__device__ __forceinline__ uint32_t derive_mask(int r, bool live) {
  const uint64_t g0 = __ballot(live && r > 0);
  const uint64_t g1 = __ballot(live && r > 1);
  const uint64_t g2 = __ballot(live && r > 2);
  uint32_t m = g0 ? 1u : 0u;
  for (int q = 0; q < 4; ++q)
    if (g1 & node_cells(1, q & 1, q >> 1)) m |= 1u << (1 + q);
  for (int ny = 0; ny < 4; ++ny)
    for (int nx = 0; nx < 4; ++nx)
      if (g2 & node_cells(2, nx, ny)) m |= 1u << bit_of(2, nx, ny);
  return m;
}

__global__ __launch_bounds__(64) void qt_pass_kernel(QtArgs a) {
  __shared__ float s_rgb[64][3];
  __shared__ float s_D[21];
  __shared__ uint32_t s_m;
  const int tile = blockIdx.x;
  const int tx = tile % a.Tw, ty = tile / a.Tw;
  const int t = threadIdx.x;
  const int cx = t & 7, cy = t >> 3;
  const int gx = tx * 8 + cx, gy = ty * 8 + cy;
  const bool live = gx < a.Cw && gy < a.Ch;
  const uint32_t pm = a.prev_mask ? a.prev_mask[tile] : 0u;

  int L;
  if (a.mode == 0) {
    // corner samples: x index 0..3 = left corners k B/4, 4..7 = right corners
    // (k+1) B/4 - 1, clamped to the frame
    {
      const int ix = t & 7, iy = t >> 3;
      const int q = a.B >> 2;
      const int ox = ix < 4 ? ix * q : (ix - 3) * q - 1;
      const int oy = iy < 4 ? iy * q : (iy - 3) * q - 1;
      const int sx = min(tx * a.B + ox, a.W - 1), sy = min(ty * a.B + oy, a.H - 1);
      const size_t pix = (size_t)sy * a.W + sx;
      s_rgb[t][0] = a.rgb[3 * pix + 0];
      s_rgb[t][1] = a.rgb[3 * pix + 1];
      s_rgb[t][2] = a.rgb[3 * pix + 2];
    }
    __syncthreads();
    if (t < 21) {
      int lvl, nx, ny;
      if (t == 0) { lvl = 0; nx = 0; ny = 0; }
      else if (t < 5) { lvl = 1; nx = (t - 1) & 1; ny = (t - 1) >> 1; }
      else { lvl = 2; nx = (t - 5) & 3; ny = (t - 5) >> 2; }
      const int span = 4 >> lvl;               // node side in units of B/4
      const int xl = nx * span, yl = ny * span;  // left / top corner index
      const int xr = 3 + xl + span, yr = 3 + yl + span;
      float D = 0.0f;
      if (tx * a.B + xl * (a.B >> 2) < a.W && ty * a.B + yl * (a.B >> 2) < a.H) {
        const int ci[4] = {yl * 8 + xl, yl * 8 + xr, yr * 8 + xl, yr * 8 + xr};
        float sum = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = u + 1; v < 4; ++v) {
            const float d0 = s_rgb[ci[u]][0] - s_rgb[ci[v]][0];
            const float d1 = s_rgb[ci[u]][1] - s_rgb[ci[v]][1];
            const float d2 = s_rgb[ci[u]][2] - s_rgb[ci[v]][2];
            sum += sqrtf(fmaf(d0, d0, fmaf(d1, d1, d2 * d2)));
          }
        D = sum / 6.0f;
      }
      s_D[bit_of(lvl, nx, ny)] = D;
    }
    __syncthreads();
    if (t == 0) {
      uint32_t m = 0;
      for (int lvl = 0; lvl <= 2; ++lvl) {
        const int n = 1 << lvl;
        for (int ny = 0; ny < n; ++ny)
          for (int nx = 0; nx < n; ++nx) {
            if (lvl > 0 && !(m & (1u << bit_of(lvl - 1, nx >> 1, ny >> 1)))) continue;
            const int bit = bit_of(lvl, nx, ny);
            const float D = s_D[bit];
            const bool split = (a.prev_mask && (pm & (1u << bit))) ? !(D < a.tau_merge) : (D > a.tau_split);
            if (split) m |= 1u << bit;
          }
      }
      s_m = m;
    }
    __syncthreads();
    L = leaf_of(s_m, cx, cy);
    if (a.prev_mask) {
      const int pl = leaf_of(pm, cx, cy);
      L = min(max(L, pl - 1), pl + 1);
    }
  } else {
    L = 0;
    if (live) {
      const size_t c = (size_t)gy * a.Cw + gx;
      const int own = a.Lin[c];
      int r = own;
      if (gx > 0) r = max(r, (int)a.Lin[c - 1] - 1);
      if (gx < a.Cw - 1) r = max(r, (int)a.Lin[c + 1] - 1);
      if (gy > 0) r = max(r, (int)a.Lin[c - a.Cw] - 1);
      if (gy < a.Ch - 1) r = max(r, (int)a.Lin[c + a.Cw] - 1);
      L = r;
    }
  }
  const uint32_t m = derive_mask(L, live);
  const int Lf = leaf_of(m, cx, cy);
  if (live) {
    const size_t c = (size_t)gy * a.Cw + gx;
    if (a.final_pass) a.level[c] = (uint8_t)Lf;
    else a.Lout[c] = (uint8_t)Lf;
  }
  if (!a.final_pass) return;
  if (t == 0) a.mask[tile] = m;
  // occupancy: a cell is occupied when some pixel inside it (and the frame)
  // has at least one fragment
  bool occ = false;
  if (live) {
    const int cs = a.B >> 3;
    const int x0 = gx * cs, y0 = gy * cs;
    const int x1 = min(x0 + cs, a.W), y1 = min(y0 + cs, a.H);
    for (int y = y0; y < y1 && !occ; ++y)
      for (int x = x0; x < x1; ++x)
        if (a.count[(size_t)y * a.W + x]) { occ = true; break; }
  }
  const uint64_t om = __ballot(occ);
  if (t == 0) {
    uint32_t h[4] = {0, 0, 0, 0};
    if (!(m & 1u)) {
      h[0] += om != 0;
    } else {
      for (int q = 0; q < 4; ++q) {
        const int qx = q & 1, qy = q >> 1;
        if (!(m & (1u << (1 + q)))) { h[1] += (om & node_cells(1, qx, qy)) != 0; continue; }
        for (int r2 = 0; r2 < 4; ++r2) {
          const int nx = 2 * qx + (r2 & 1), ny = 2 * qy + (r2 >> 1);
          const uint64_t cells = node_cells(2, nx, ny);
          if (!(m & (1u << bit_of(2, nx, ny)))) { h[2] += (om & cells) != 0; continue; }
          h[3] += __popcll(om & cells);
        }
      }
    }
    for (int l = 0; l < 4; ++l) a.tile_hist[4 * (size_t)tile + l] = h[l];
  }
}

struct FinishArgs {
  int W, H, T;
  const uint32_t* tile_hist;
  starnt_sched* sched;
};

__global__ __launch_bounds__(64) void qt_finish_kernel(FinishArgs a) {
  const int t = threadIdx.x;
  uint32_t h[4] = {0, 0, 0, 0};
  for (int i = t; i < a.T; i += 64)
    for (int l = 0; l < 4; ++l) h[l] += a.tile_hist[4 * (size_t)i + l];
  for (int off = 32; off > 0; off >>= 1)
    for (int l = 0; l < 4; ++l) h[l] += __shfl_down(h[l], off);
  if (t == 0) {
    starnt_sched* s = a.sched;
    const double den = (double)h[0] + h[1] + h[2] + h[3];
    const double wb = den > 0 ? ((double)h[1] + 2.0 * h[2] + 3.0 * h[3]) / den : 0.0;
    const double s2 = fmin(1.0, fmax(0.25, exp2(wb - 2.2)));
    const double s3 = fmin(1.0, fmax(0.25, exp2(wb - 3.0)));
    auto dim = [](int n, double sc) {
      double v = ceil(sc * (double)n);
      v = fmax(1.0, fmin((double)n, v));
      return (int)v;
    };
    for (int l = 0; l < 4; ++l) s->hist[l] = h[l];
    s->wbar = (float)wb;
    s->s2 = (float)s2;
    s->s3 = (float)s3;
    s->w2 = dim(a.W, s2);
    s->h2 = dim(a.H, s2);
    s->w3 = dim(a.W, s3);
    s->h3 = dim(a.H, s3);
    s->frames = s->frames + 1;
  }
}

struct InitArgs {
  starnt_sched* s;
  int w2, h2, w3, h3;
};

__global__ void sched_init_kernel(InitArgs a) {
  starnt_sched* s = a.s;
  s->w2 = a.w2; s->h2 = a.h2; s->w3 = a.w3; s->h3 = a.h3;
  for (int l = 0; l < 4; ++l) s->hist[l] = 0;
  s->wbar = 0.0f; s->s2 = 1.0f; s->s3 = 1.0f;
  s->frames = 0;
  for (int i = 0; i < 4; ++i) s->pad[i] = 0;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

size_t quadtree_ws_bytes(int64_t W, int64_t H, int64_t B) {
  if (W <= 0 || H <= 0 || B < 8 || (B & 7)) return 0;
  const int64_t cs = B / 8;
  const int64_t Cw = (W + cs - 1) / cs, Ch = (H + cs - 1) / cs;
  const int64_t T = ((W + B - 1) / B) * ((H + B - 1) / B);
  return 2 * align256((size_t)(Cw * Ch)) + align256((size_t)T * 16);
}

int launch_quadtree(const float* rgb, const uint32_t* count, int W, int H, const starnt_qt_params& qp,
                    const uint32_t* prev_mask, uint32_t* mask, uint8_t* level, starnt_sched* sched, void* ws,
                    hipStream_t s) {
  QtArgs a;
  a.W = W; a.H = H; a.B = qp.base;
  a.Tw = (W + qp.base - 1) / qp.base;
  a.Th = (H + qp.base - 1) / qp.base;
  const int cs = qp.base / 8;
  a.Cw = (W + cs - 1) / cs;
  a.Ch = (H + cs - 1) / cs;
  a.tau_split = qp.tau_split;
  a.tau_merge = qp.tau_merge;
  a.rgb = rgb;
  a.count = count;
  a.prev_mask = prev_mask;
  a.mask = mask;
  a.level = level;
  uint8_t* L0 = static_cast<uint8_t*>(ws);
  uint8_t* L1 = L0 + align256((size_t)a.Cw * a.Ch);
  a.tile_hist = reinterpret_cast<uint32_t*>(L1 + align256((size_t)a.Cw * a.Ch));
  const int T = a.Tw * a.Th;
  uint8_t* bufs[2] = {L0, L1};
  for (int it = 0; it <= qp.k_relax; ++it) {
    a.mode = it == 0 ? 0 : 1;
    a.final_pass = it == qp.k_relax;
    a.Lin = bufs[(it + 1) & 1];
    a.Lout = bufs[it & 1];
    hipLaunchKernelGGL(qt_pass_kernel, dim3(T), dim3(64), 0, s, a);
    STARNT_LAUNCH_CHECK("starnt_quadtree pass launch");
  }
  FinishArgs f;
  f.W = W; f.H = H; f.T = T;
  f.tile_hist = a.tile_hist;
  f.sched = sched;
  hipLaunchKernelGGL(qt_finish_kernel, dim3(1), dim3(64), 0, s, f);
  STARNT_LAUNCH_CHECK("starnt_quadtree finish launch");
  return STARNT_OK;
}

int launch_sched_init(starnt_sched* sched, int w2, int h2, int w3, int h3, hipStream_t s) {
  InitArgs a{sched, w2, h2, w3, h3};
  hipLaunchKernelGGL(sched_init_kernel, dim3(1), dim3(1), 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_sched_init launch");
  return STARNT_OK;
}

}  // namespace starnt
