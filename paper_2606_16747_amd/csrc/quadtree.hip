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
//  one-block kernel sums them and computes wbar, s2, s3 and the next grids on
//  the device.
#include <mutex>

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
  uint64_t* tile_occ;   // [T] occupied cells, from the top-down pass
  int mode;             // 0 top-down, 1 relaxation
  int final_pass;
};

// Sum of the per-tile leaf counts and the schedule they imply (eq (4)), by
// the 64 threads of one block. Integer sums: exact in any order.
__device__ void finish_schedule(const uint32_t* tile_hist, int T, int W, int H, starnt_sched* s, int t) {
  uint32_t h[4] = {0, 0, 0, 0};
  const uint4* th = reinterpret_cast<const uint4*>(tile_hist);  // 256-byte aligned
  for (int i0 = 0; i0 < T; i0 += 64 * 8) {
    uint4 v[8];  // eight loads in flight per thread
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + 64 * u + t;
      v[u] = i < T ? th[i] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      h[0] += v[u].x; h[1] += v[u].y; h[2] += v[u].z; h[3] += v[u].w;
    }
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int l = 0; l < 4; ++l) h[l] += __shfl_down(h[l], off);
  if (t == 0) {
    // FP32 (a grid side can differ from the FP64 definition only where
    // s * n lies within FP32 rounding of an integer)
    const float den = (float)h[0] + (float)h[1] + (float)h[2] + (float)h[3];
    const float wb = den > 0.0f ? ((float)h[1] + 2.0f * (float)h[2] + 3.0f * (float)h[3]) / den : 0.0f;
    const float s2 = fminf(1.0f, fmaxf(0.25f, exp2f(wb - 2.2f)));
    const float s3 = fminf(1.0f, fmaxf(0.25f, exp2f(wb - 3.0f)));
    auto dim = [](int n, float sc) {
      float v = ceilf(sc * (float)n);
      v = fmaxf(1.0f, fminf((float)n, v));
      return (int)v;
    };
    for (int l = 0; l < 4; ++l) s->hist[l] = h[l];
    s->wbar = wb;
    s->s2 = s2;
    s->s3 = s3;
    s->w2 = dim(W, s2);
    s->h2 = dim(H, s2);
    s->w3 = dim(W, s3);
    s->h3 = dim(H, s3);
    s->frames = s->frames + 1;
  }
}

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

// Occupied cells of a tile as a 64-bit mask (bit 8 cy + cx): a cell is
// occupied when some pixel inside it (and the frame) has at least one
// fragment. Called by all 64 threads of the tile's block.
__device__ __forceinline__ uint64_t tile_occupancy(const QtArgs& a, int tx, int ty, int t, int gx, int gy,
                                                   bool live) {
  uint64_t om;
  if (a.B == 64) {
    // lane = pixel column of the tile; each row is one coalesced 256-byte
    // load, OR-ed per 8-row band; a cell's 8 columns are 8 bits of a ballot
    // (addresses are clamped into the frame and values outside it dropped,
    // so the 64 loads carry no branches and are all in flight together)
    const int px = tx * 64 + t;
    const bool col_in = px < a.W;
    const uint32_t* col = a.count + min(px, a.W - 1);
    const int rows = min(64, a.H - ty * 64);  // rows of the tile inside the frame
    uint32_t v[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) v[r] = col[(size_t)(ty * 64 + min(r, rows - 1)) * a.W];
    uint32_t band = 0;  // bit cy: this column has a fragment in cell row cy
#pragma unroll
    for (int cy8 = 0; cy8 < 8; ++cy8) {
      uint32_t any = 0;
#pragma unroll
      for (int dy = 0; dy < 8; ++dy) any |= v[8 * cy8 + dy];  // rows past the frame repeat the last
      band |= (any != 0 ? 1u : 0u) << cy8;
    }
    // cell rows past the frame are empty; so are columns past it
    band &= rows >= 64 ? 0xFFu : ((1u << ((rows + 7) >> 3)) - 1u);
    band = col_in ? band : 0u;
    om = 0;
#pragma unroll
    for (int cy8 = 0; cy8 < 8; ++cy8) {
      const uint64_t cols = __ballot((band >> cy8) & 1u);
#pragma unroll
      for (int cx8 = 0; cx8 < 8; ++cx8)
        if ((cols >> (8 * cx8)) & 0xFFull) om |= 1ull << (8 * cy8 + cx8);
    }
  } else {
    bool occ = false;
    if (live) {
      const int cs = a.B >> 3;
      const int x0 = gx * cs, y0 = gy * cs;
      const int x1 = min(x0 + cs, a.W), y1 = min(y0 + cs, a.H);
      uint32_t any = 0;
      for (int y = y0; y < y1; ++y)
#pragma unroll 8
        for (int x = x0; x < x1; ++x) any |= a.count[(size_t)y * a.W + x];
      occ = any != 0;
    }
    om = __ballot(occ);
  }
  return om;
}

__device__ void write_final(const QtArgs& a, int tile, int t, uint32_t m, int Lf, bool live, int gx, int gy);

__global__ __launch_bounds__(64) void qt_pass_kernel(QtArgs a) {
  __shared__ float s_rgb[64][3];
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
    // (k+1) B/4 - 1, clamped to the frame; lane t loads sample t
    float cr, cg, cb;
    {
      const int ix = t & 7, iy = t >> 3;
      const int q = a.B >> 2;
      const int ox = ix < 4 ? ix * q : (ix - 3) * q - 1;
      const int oy = iy < 4 ? iy * q : (iy - 3) * q - 1;
      const int sx = min(tx * a.B + ox, a.W - 1), sy = min(ty * a.B + oy, a.H - 1);
      const size_t pix = (size_t)sy * a.W + sx;
      cr = a.rgb[3 * pix + 0];
      cg = a.rgb[3 * pix + 1];
      cb = a.rgb[3 * pix + 2];
    }
    // cell occupancy for the histogram of the last pass (its loads are in
    // flight together with the corner sample's)
    const uint64_t om = tile_occupancy(a, tx, ty, t, gx, gy, live);
    if (t == 0) a.tile_occ[tile] = om;
    s_rgb[t][0] = cr;
    s_rgb[t][1] = cg;
    s_rgb[t][2] = cb;
    __syncthreads();
    // lane t < 21 evaluates node bit t (0 root; 1..4 level 1; 5..20 level 2,
    // quadrant-major): its D and its own split/merge decision with
    // hysteresis; the decisions are gathered with a ballot and gated top-down
    // (a node counts only under a split parent)
    bool own_split = false;
    if (t < 21) {
      int lvl, nx, ny;
      if (t == 0) { lvl = 0; nx = 0; ny = 0; }
      else if (t < 5) { lvl = 1; nx = (t - 1) & 1; ny = (t - 1) >> 1; }
      else {
        const int q = (t - 5) >> 2, r = (t - 5) & 3;
        lvl = 2; nx = 2 * (q & 1) + (r & 1); ny = 2 * (q >> 1) + (r >> 1);
      }
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
      own_split = (a.prev_mask && (pm & (1u << t))) ? !(D < a.tau_merge) : (D > a.tau_split);
    }
    const uint32_t own = (uint32_t)__ballot(own_split);
    const uint32_t m0 = own & 1u;
    const uint32_t m1 = m0 ? (own & 0x1Eu) : 0u;
    uint32_t m2 = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if ((m1 >> (1 + q)) & 1u) m2 |= own & (0xFu << (5 + 4 * q));
    const uint32_t mtd = m0 | m1 | m2;
    L = leaf_of(mtd, cx, cy);
    if (a.prev_mask) {
      const int pl = leaf_of(pm, cx, cy);
      L = min(max(L, pl - 1), pl + 1);
    }
  } else {
    // own level and the 4 neighbours' (clamped to the grid: a clamped
    // neighbour is the cell itself, which cannot raise it), loads issued
    // together
    const int cxl = min(gx, a.Cw - 1), cyl = min(gy, a.Ch - 1);
    const size_t c = (size_t)cyl * a.Cw + cxl;
    const int own = a.Lin[c];
    const int l = a.Lin[(size_t)cyl * a.Cw + max(cxl - 1, 0)];
    const int rr = a.Lin[(size_t)cyl * a.Cw + min(cxl + 1, a.Cw - 1)];
    const int u = a.Lin[(size_t)max(cyl - 1, 0) * a.Cw + cxl];
    const int d = a.Lin[(size_t)min(cyl + 1, a.Ch - 1) * a.Cw + cxl];
    L = live ? max(max(own, max(l, rr) - 1), max(u, d) - 1) : 0;
  }
  const uint32_t m = derive_mask(L, live);
  const int Lf = leaf_of(m, cx, cy);
  if (a.final_pass) {
    write_final(a, tile, t, m, Lf, live, gx, gy);
  } else if (live) {
    a.Lout[(size_t)gy * a.Cw + gx] = (uint8_t)Lf;
  }
}

// the last pass's outputs for one tile: leaf levels, the mask and the
// tile's occupied-leaf counts per level (lane t = cell t)
__device__ void write_final(const QtArgs& a, int tile, int t, uint32_t m, int Lf, bool live, int gx, int gy) {
  if (live) a.level[(size_t)gy * a.Cw + gx] = (uint8_t)Lf;
  if (t == 0) a.mask[tile] = m;
  const uint64_t om = a.tile_occ[tile];
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

// Both relaxations (k = 2) in one launch. A block of nine waves takes one
// tile: wave w runs the first relaxation for tile (tx + w % 3 - 1,
// ty + w / 3 - 1) of its 3 x 3 neighbourhood from the top-down levels, into
// LDS; the centre wave then runs the second relaxation, whose cells' 4
// neighbours all lie in that neighbourhood, and writes the outputs. The first
// relaxation of a tile depends only on the top-down levels, so each block's
// copies equal what a separate pass would write. Integer work, identical.
__global__ __launch_bounds__(576) void qt_relax2_kernel(QtArgs a) {
  __shared__ uint8_t s_lv[9][64];
  const int tile = blockIdx.x;
  const int tx = tile % a.Tw, ty = tile / a.Tw;
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int cx = t & 7, cy = t >> 3;
  // ---- first relaxation, one neighbourhood tile per wave ----
  {
    const int nx = tx + w % 3 - 1, ny = ty + w / 3 - 1;
    if (nx >= 0 && nx < a.Tw && ny >= 0 && ny < a.Th) {  // uniform over the wave
      const int gx = nx * 8 + cx, gy = ny * 8 + cy;
      const bool live = gx < a.Cw && gy < a.Ch;
      const int cxl = min(gx, a.Cw - 1), cyl = min(gy, a.Ch - 1);
      const int own = a.Lin[(size_t)cyl * a.Cw + cxl];
      const int l = a.Lin[(size_t)cyl * a.Cw + max(cxl - 1, 0)];
      const int rr = a.Lin[(size_t)cyl * a.Cw + min(cxl + 1, a.Cw - 1)];
      const int u = a.Lin[(size_t)max(cyl - 1, 0) * a.Cw + cxl];
      const int d = a.Lin[(size_t)min(cyl + 1, a.Ch - 1) * a.Cw + cxl];
      const int L = live ? max(max(own, max(l, rr) - 1), max(u, d) - 1) : 0;
      s_lv[w][t] = (uint8_t)leaf_of(derive_mask(L, live), cx, cy);
    }
  }
  __syncthreads();
  if (w != 4) return;
  // ---- second relaxation of the centre tile ----
  const int gx = tx * 8 + cx, gy = ty * 8 + cy;
  const bool live = gx < a.Cw && gy < a.Ch;
  const int cxl = min(gx, a.Cw - 1), cyl = min(gy, a.Ch - 1);
  // level of in-grid cell (x, y), which lies in the neighbourhood
  auto at = [&](int x, int y) -> int {
    const int sw = (x >> 3) - tx + 1, sh = (y >> 3) - ty + 1;
    return s_lv[sh * 3 + sw][(y & 7) * 8 + (x & 7)];
  };
  const int own = at(cxl, cyl);
  const int l = at(max(cxl - 1, 0), cyl);
  const int rr = at(min(cxl + 1, a.Cw - 1), cyl);
  const int u = at(cxl, max(cyl - 1, 0));
  const int d = at(cxl, min(cyl + 1, a.Ch - 1));
  const int L = live ? max(max(own, max(l, rr) - 1), max(u, d) - 1) : 0;
  const uint32_t m = derive_mask(L, live);
  write_final(a, tile, t, m, leaf_of(m, cx, cy), live, gx, gy);
}

// one block: the schedule of the next frame from all tiles' counts
__global__ __launch_bounds__(64) void qt_finish_kernel(const uint32_t* tile_hist, int T, int W, int H,
                                                       starnt_sched* sched) {
  finish_schedule(tile_hist, T, W, H, sched, threadIdx.x);
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
  return 2 * align256((size_t)(Cw * Ch)) + align256((size_t)T * 16) + align256((size_t)T * 8);
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
  a.tile_occ = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(a.tile_hist) + align256((size_t)T * 16));
  uint8_t* bufs[2] = {L0, L1};
  // k = 2 (the usual setting): the top-down pass, then both relaxations in
  // one launch; otherwise one launch per pass
  const int passes = qp.k_relax == 2 ? 1 : qp.k_relax;
  for (int it = 0; it <= passes; ++it) {
    a.mode = it == 0 ? 0 : 1;
    a.final_pass = it == qp.k_relax;
    a.Lin = bufs[(it + 1) & 1];
    a.Lout = bufs[it & 1];
    if (qp.k_relax == 2 && it == 1) {
      a.final_pass = 1;
      hipLaunchKernelGGL(qt_relax2_kernel, dim3(T), dim3(576), 0, s, a);
    } else {
      hipLaunchKernelGGL(qt_pass_kernel, dim3(T), dim3(64), 0, s, a);
    }
    STARNT_LAUNCH_CHECK("starnt_quadtree pass launch");
  }
  hipLaunchKernelGGL(qt_finish_kernel, dim3(1), dim3(64), 0, s, a.tile_hist, T, W, H, sched);
  STARNT_LAUNCH_CHECK("starnt_quadtree finish launch");
  return STARNT_OK;
}

int launch_sched_init(starnt_sched* sched, int w2, int h2, int w3, int h3, hipStream_t s) {
  InitArgs a{sched, w2, h2, w3, h3};
  hipLaunchKernelGGL(sched_init_kernel, dim3(1), dim3(1), 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_sched_init launch");
  return STARNT_OK;
}

// Scratch of the allocation-free quadtree update: a fixed array in device
// memory (each GPU the library runs on holds its own copy until the process
// ends). Host code never passes the array's name to a kernel: in host code it
// is only a handle, and the device address of the current GPU's copy comes
// from hipGetSymbolAddress, resolved once per device.
constexpr size_t kQtScratchBytes = size_t(4) << 20;
static __device__ __align__(256) uint8_t scratch[kQtScratchBytes];

size_t quadtree_scratch_bytes() { return kQtScratchBytes; }

int launch_quadtree_noalloc(const float* rgb, const uint32_t* count, int W, int H, const starnt_qt_params& qp,
                            const uint32_t* prev_mask, uint32_t* mask, uint8_t* level, starnt_sched* sched,
                            hipStream_t s) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  const size_t need = quadtree_ws_bytes(W, H, qp.base);
  if (need > kQtScratchBytes)
    return fail(STARNT_ENOMEM, "starnt_quadtree_noalloc: this frame and base need " + std::to_string(need) +
                                   " bytes of scratch; the allocation-free call holds " +
                                   std::to_string(kQtScratchBytes) + " (use starnt_quadtree with a workspace)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "starnt_quadtree_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(STARNT_EUNSUPPORTED, "starnt_quadtree_noalloc: device index above 63");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
      // with `dev` current: the address of this GPU's copy of the array
      e = hipGetSymbolAddress(&addr[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        addr[dev] = nullptr;
        return hip_status(e, "starnt_quadtree_noalloc: hipGetSymbolAddress(scratch)");
      }
    }
    ptr = addr[dev];
  }
  return launch_quadtree(rgb, count, W, H, qp, prev_mask, mask, level, sched, ptr, s);
}

}  // namespace starnt
