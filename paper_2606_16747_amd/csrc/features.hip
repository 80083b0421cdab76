// Passes 1-3 of STAR-NT (Sec. 3, Fig. 1) over per-pixel fragment lists.
//
// Per pixel:
//  * pass 1 (every pixel): nearest fragment by (depth, prim) -> d1, layer 1, N;
//  * pass 2 (pixels sampled by the pass-2 grid): second-nearest -> layer 2;
//  * pass 3 (pixels sampled by the pass-3 grid): order-independent sums over
//    ALL fragments in exact fixed point, then the two selected layers are
//    subtracted exactly, leaving the tail (sorted positions 3..N):
//      A = sum a, S = sum a c (a c rounded once in FP32), Lg = sum -log2(1 - a),
//    giving x = (N, t_tail = 2^-Lg, Ct = S / A) (Sec. 3.3).
// Integer sums make every output independent of the order of a list.
// Scales: A and S in Q24, Lg in Q27 in 64 bits; an opaque fragment (a = 1)
// adds 2^36 to Lg, so 2^-Lg is exactly 0 while it is in the tail and the
// exact subtraction removes it when it is a selected layer. Lists of up to
// 255 fragments keep A and S in 32 bits end to end; a wave holding a longer
// list takes a 64-bit variant (lane-local 32-bit partials folded into 64 bits
// every 128 steps), chosen once per wave.
//
// Memory layout of the work: four lanes own a pixel and stride through its
// list together, so every load instruction of a quad covers a contiguous run
// of the CSR arrays (16 B of depth, 64 B of RGBA) that is consumed at once;
// a wave streams 16 neighbouring pixels, whose lists are adjacent in memory.
// A row off the pass-3 grid streams depths only (no colour loads, no sums);
// on a row of the grid, pixels off it skip their RGBA loads inside the same
// loop (their terms are zero), so a wave never runs two loop variants.
// No LDS and no barriers: the per-lane partial state (top-2 keys, fixed-point
// sums) is merged across the quad with DPP quad permutations; after the
// merge each lane of the quad finishes one colour channel.
//
// The kernel runs near the copy rate of HBM with its VALU busy most of the
// time, and each wave waits on a short chain of dependent loads (offsets,
// then the fragments, then the two selected colours). Per-fragment work is
// kept to straight-line compares, selects and one-instruction roundings.
// Measured at 1080p, neither fewer instructions per pixel (a one-lane finish)
// nor more loads in flight per lane (four fragments per step) was faster:
// both lengthened a wave's chain or cost occupancy.
#include "internal.h"

namespace starnt {
namespace {

constexpr float kQ24 = 16777216.0f;     // 2^24
constexpr float kQ27 = 134217728.0f;    // 2^27
constexpr uint64_t kOpaque = 1ull << 36;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kOne = 0x3F800000u;  // bits of 1.0f
constexpr int kG = 4;                   // lanes per pixel
constexpr uint32_t kNarrow = 255;       // longest list with 32-bit channel sums
constexpr uint32_t kFold = 128;         // lane steps between 32 -> 64-bit folds

// Quad permutations (DPP quad_perm, lane i reads lane perm[i] of its quad).
constexpr int kXor1 = 0xB1;  // [1,0,3,2]
constexpr int kXor2 = 0x4E;  // [2,3,0,1]
constexpr int kRot1 = 0x39;  // [1,2,3,0]
constexpr int kBc0 = 0x00;   // [0,0,0,0]
template <int CTRL>
__device__ __forceinline__ uint32_t qperm(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float qperm(float v) {
  return __uint_as_float(qperm<CTRL>(__float_as_uint(v)));
}
template <int CTRL>
__device__ __forceinline__ uint64_t qperm(uint64_t v) {
  return (uint64_t)qperm<CTRL>((uint32_t)v) | ((uint64_t)qperm<CTRL>((uint32_t)(v >> 32)) << 32);
}

struct FeatArgs {
  int W, H;
  const uint32_t* off;
  const float* depth;
  const void* rgba;
  const uint32_t* prim;
  uint32_t max_n;
  const starnt_sched* sched;
  float* d1;
  float4* layer1;
  uint32_t* count;
  float4* layer2;
  float4* tail;
  uint2* sel;
  uint32_t* err;
  float4* tail_avg;  // optional tail means (DFAOIT inputs)
  const uint32_t* list;    // listed pixels (patch only)
  const uint32_t* list_n;  // number of listed pixels (patch only)
  uint32_t frame_p;        // pixels of the frame the list indexes (patch only)
};

// Fixed-point terms of one fragment. Each is an exact integer function of
// its fragment, so the sums stay order independent. Q24 terms round half up
// (floor(x + 1/2), one instruction; unbiased but for exact halves, so the
// error of a sum grows with the square root of its length); they are at
// most 2^24 for colours in [0, 1].
__device__ __forceinline__ uint32_t round_q(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return (uint32_t)r;
}
__device__ __forceinline__ uint64_t lg_term(float a) {
  const float l = -__log2f(1.0f - a) * kQ27;  // <= 24 * 2^27 below a = 1
  return a >= 1.0f ? kOpaque : (uint64_t)(uint32_t)__builtin_rintf(l);
}
struct Terms {
  uint32_t a, r, g, b;
  uint64_t lg;
};
__device__ __forceinline__ Terms frag_terms(float4 c) {
  Terms t;
  const float a = __builtin_amdgcn_fmed3f(c.w, 0.0f, 1.0f);
  const float a24 = a * kQ24;  // exact scaling: a24 * c = (a * c) * 2^24
  t.a = round_q(a24);
  t.r = round_q(a24 * c.x);
  t.g = round_q(a24 * c.y);
  t.b = round_q(a24 * c.z);
  t.lg = lg_term(a);
  return t;
}

// channel sums: V is uint32_t for lists of at most kNarrow fragments, else
// uint64_t (then fed from 32-bit lane partials folded every kFold steps)
template <typename V>
struct Sums {
  V a = 0, r = 0, g = 0, b = 0;
  V cr = 0, cg = 0, cb = 0;  // plain colour sums (tail means only)
  uint64_t lg = 0;
};
struct Part {
  uint32_t a = 0, r = 0, g = 0, b = 0;
  uint32_t cr = 0, cg = 0, cb = 0;
};
template <bool AVG, typename V>
__device__ __forceinline__ void fold(Sums<V>& s, Part& p) {
  s.a += p.a; s.r += p.r; s.g += p.g; s.b += p.b;
  if (AVG) { s.cr += p.cr; s.cg += p.cg; s.cb += p.cb; }
  p = Part();
}

// two smallest (depth, prim) keys; prim is read only on equal depths
struct Top2 {
  float z1 = __builtin_inff(), z2 = __builtin_inff();
  uint32_t k1 = kNone, k2 = kNone;  // global fragment indices
};

// Insert key (z, k) into the top 2. The common case is two compares and four
// selects; an exact depth tie with a held key (rare) loads primitive ids for
// the tie-break. A NaN depth never enters (every compare is false), and
// neither does a key at the empty slots' +inf depth.
__device__ __forceinline__ void top2_push(Top2& t, float z, uint32_t k, const uint32_t* prim) {
  bool lt1 = z < t.z1, lt2 = z < t.z2;
  if (z == t.z1 || z == t.z2) {
    const bool eq1 = z == t.z1 && t.k1 != kNone && k != kNone;
    const bool eq2 = z == t.z2 && t.k2 != kNone && k != kNone;
    if (eq1 || eq2) {
      const uint32_t pk = prim[k];
      if (eq1) lt1 = pk < prim[t.k1];
      if (eq2) lt2 = pk < prim[t.k2];
    }
  }
  t.z2 = lt1 ? t.z1 : (lt2 ? z : t.z2);
  t.k2 = lt1 ? t.k1 : (lt2 ? k : t.k2);
  t.z1 = lt1 ? z : t.z1;
  t.k1 = lt1 ? k : t.k1;
}

template <bool AVG>
__device__ __forceinline__ void add_terms(Part& p, uint64_t& lg, const Terms& q, float4 c) {
  p.a += q.a; p.r += q.r; p.g += q.g; p.b += q.b;
  lg += q.lg;
  if (AVG) {  // plain colour in Q24 (a colour is zero when its fragment is absent)
    p.cr += round_q(c.x * kQ24);
    p.cg += round_q(c.y * kQ24);
    p.cb += round_q(c.z * kQ24);
  }
}

// Depth-only stream for rows off the pass-3 grid: the top-2 keys and the
// depth check, with no colour loads and no sums.
__device__ __forceinline__ void stream_depth(const FeatArgs& a, uint32_t b, uint32_t e, int q, Top2& t,
                                             uint32_t& zmax) {
  uint32_t k = b + q;
  for (; k + kG < e; k += 2 * kG) {
    const float z0 = a.depth[k], z1 = a.depth[k + kG];
    zmax = max(zmax, max(__float_as_uint(z0), __float_as_uint(z1)));
    top2_push(t, z0, k, a.prim);
    top2_push(t, z1, k + kG, a.prim);
  }
  if (k < e) {
    const float z = a.depth[k];
    zmax = max(zmax, __float_as_uint(z));
    top2_push(t, z, k, a.prim);
  }
}

// One lane's share of a list: fragments b+q, b+q+4, ..., two per step so both
// loads are in flight together. RGBA is loaded only when `rgba` (pass-3
// pixels); otherwise the colour is zero and so are its terms.
template <bool HALF, bool WIDE, bool AVG, typename V>
__device__ __forceinline__ void stream(const FeatArgs& a, uint32_t b, uint32_t e, int q, bool rgba, Top2& t,
                                       Sums<V>& s, uint32_t& zmax, uint32_t& amax) {
  Part p;
  uint32_t k = b + q;
  // colours stay zero in lanes that never load them (rgba is per pixel)
  float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
  do {
    const uint32_t kend = WIDE ? min(e, k + kFold * kG) : e;
    for (; k + kG < kend; k += 2 * kG) {
      const float z0 = a.depth[k], z1 = a.depth[k + kG];
      if (rgba) {
        c0 = load_rgba<HALF>(a.rgba, k);
        c1 = load_rgba<HALF>(a.rgba, k + kG);
      }
      zmax = max(zmax, max(__float_as_uint(z0), __float_as_uint(z1)));  // -0, negatives, NaN exceed 1.0's bits
      top2_push(t, z0, k, a.prim);
      top2_push(t, z1, k + kG, a.prim);
      amax = max(amax, max(__float_as_uint(c0.w), __float_as_uint(c1.w)));
      add_terms<AVG>(p, s.lg, frag_terms(c0), c0);
      add_terms<AVG>(p, s.lg, frag_terms(c1), c1);
    }
    if (k < kend) {
      const float z = a.depth[k];
      if (rgba) c0 = load_rgba<HALF>(a.rgba, k);
      zmax = max(zmax, __float_as_uint(z));
      top2_push(t, z, k, a.prim);
      amax = max(amax, __float_as_uint(c0.w));
      add_terms<AVG>(p, s.lg, frag_terms(c0), c0);
      k += kG;
    }
    fold<AVG>(s, p);
  } while (WIDE && k < e);
}

// channel sum -> FP32
__device__ __forceinline__ float to_f32(uint32_t v) { return (float)v; }
__device__ __forceinline__ float to_f32(uint64_t v) {
  return __builtin_fmaf((float)(uint32_t)(v >> 32), 4294967296.0f, (float)(uint32_t)v);
}
// 2^(-Lg / 2^27): an opaque fragment (2^36) or any Lg of 2^36 and above gives
// exactly 0; below that Lg / 2^27 = 32 hi + lo / 2^27
__device__ __forceinline__ float tail_transmittance(uint64_t lg) {
  const uint32_t hi = (uint32_t)(lg >> 32), lo = (uint32_t)lg;
  const float e = __builtin_fmaf((float)hi, 32.0f, (float)lo * (1.0f / kQ27));
  return hi >= 16u ? 0.0f : __builtin_amdgcn_exp2f(-e);
}

// SUMS = false: the pixel's row is off the pass-3 grid (depth-only stream).
template <bool HALF, bool WIDE, bool AVG, bool SUMS>
__device__ __forceinline__ void pixel(const FeatArgs& a, const Grids& g, int p, int q, uint32_t b, uint32_t e,
                                      int i2, int j2, int i3, int j3) {
  using V = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  const bool pass2 = i2 >= 0 && j2 >= 0;
  const bool pass3 = SUMS && i3 >= 0 && j3 >= 0;
  const uint32_t n = e - b;
  Top2 t;
  Sums<V> s;
  uint32_t zmax = 0, amax = 0;
  if constexpr (SUMS) stream<HALF, WIDE, AVG>(a, b, e, q, pass3, t, s, zmax, amax);
  else stream_depth(a, b, e, q, t, zmax);

  // merge the quad's top-2 keys: two butterfly rounds
  {
    const float oz1 = qperm<kXor1>(t.z1), oz2 = qperm<kXor1>(t.z2);
    const uint32_t ok1 = qperm<kXor1>(t.k1), ok2 = qperm<kXor1>(t.k2);
    top2_push(t, oz1, ok1, a.prim);
    top2_push(t, oz2, ok2, a.prim);
  }
  {
    const float oz1 = qperm<kXor2>(t.z1), oz2 = qperm<kXor2>(t.z2);
    const uint32_t ok1 = qperm<kXor2>(t.k1), ok2 = qperm<kXor2>(t.k2);
    top2_push(t, oz1, ok1, a.prim);
    top2_push(t, oz2, ok2, a.prim);
  }
  // the two selected layers, fetched by every lane of the quad (one
  // transaction per address)
  const bool want2 = pass2 || pass3;
  float4 c1 = make_float4(0.f, 0.f, 0.f, 0.f), c2 = c1;
  if (t.k1 != kNone) c1 = load_rgba<HALF>(a.rgba, t.k1);
  if (t.k2 != kNone && want2) c2 = load_rgba<HALF>(a.rgba, t.k2);
  amax = max(amax, max(__float_as_uint(c1.w), __float_as_uint(c2.w)));

  // layer outputs (premultiplied): lane 0 -> layer 1, lane 1 -> layer 2
  {
    const float4 c = q == 0 ? c1 : c2;
    const float al = __builtin_amdgcn_fmed3f(c.w, 0.0f, 1.0f);
    if (q == 0 || (q == 1 && pass2)) {
      float4* dst = q == 0 ? a.layer1 + p : a.layer2 + (j2 * g.w2 + i2);
      *dst = make_float4(al * c.x, al * c.y, al * c.z, al);
    }
  }
  // lane 2 -> d1, lane 3 -> N
  if (q >= 2) {
    uint32_t* dst = q == 2 ? reinterpret_cast<uint32_t*>(a.d1) + p : a.count + p;
    *dst = q == 2 ? __float_as_uint(n ? t.z1 : 1.0f) : n;
  }
  if (a.sel && q == 0) a.sel[p] = make_uint2(t.k1, t.k2);

  if (SUMS && pass3) {
    // reduce-scatter of the channel sums (alpha, r, g, b): lane q ends with
    // the quad total of channel q; the log-transmittance sum is all-reduced
    const bool hi = q & 2, odd = q & 1;
    const V y0 = (hi ? s.g : s.a) + qperm<kXor2>(hi ? s.a : s.g);
    const V y1 = (hi ? s.b : s.r) + qperm<kXor2>(hi ? s.r : s.b);
    V v = (odd ? y1 : y0) + qperm<kXor1>(odd ? y0 : y1);
    uint64_t lg = s.lg + qperm<kXor1>(s.lg);
    lg += qperm<kXor2>(lg);
    // exact removal of the two selected layers leaves the tail (a missing
    // layer is all zero, so its terms are zero)
    const float m1 = q == 0 ? 1.0f : (q == 1 ? c1.x : (q == 2 ? c1.y : c1.z));
    const float m2 = q == 0 ? 1.0f : (q == 1 ? c2.x : (q == 2 ? c2.y : c2.z));
    const float a1 = __builtin_amdgcn_fmed3f(c1.w, 0.0f, 1.0f), a2 = __builtin_amdgcn_fmed3f(c2.w, 0.0f, 1.0f);
    v -= (V)round_q(a1 * kQ24 * m1);
    v -= (V)round_q(a2 * kQ24 * m2);
    lg -= lg_term(a1) + lg_term(a2);
    // x = (N, t_tail, Ct = S / A) and A, one channel per lane
    const bool tail = n > 2;
    const float tv = to_f32(v);
    const float A = qperm<kBc0>(tv);
    const float inv = (tail && A > 0.0f) ? __builtin_amdgcn_rcpf(A) : 0.0f;
    const float o = q == 0 ? (tail ? A * (1.0f / kQ24) : 0.0f) : tv * inv;
    const float tt = tail ? tail_transmittance(lg) : 1.0f;
    // record [N, t_tail, Cr, Cg | Cb, A, T2, 0] as one float2 per lane, with
    // T2 = (1 - a1)(1 - a2) the transmittance behind the two selected layers
    const float nx = qperm<kRot1>(o), oa = qperm<kBc0>(o);
    float2 rec;
    rec.x = q == 0 ? (float)n : (q == 1 ? o : (q == 2 ? nx : (1.0f - a1) * (1.0f - a2)));
    rec.y = q == 0 ? tt : (q == 1 ? nx : (q == 2 ? oa : 0.0f));
    reinterpret_cast<float2*>(a.tail + 2 * (size_t)(j3 * g.w3 + i3))[q] = rec;
    if (AVG) {
      // tail means: the colour sums all-reduced, the selected layers removed
      // exactly; lane q < 3 writes colour channel q, lane 3 the mean opacity
      V cr = s.cr + qperm<kXor1>(s.cr), cg = s.cg + qperm<kXor1>(s.cg), cb = s.cb + qperm<kXor1>(s.cb);
      cr += qperm<kXor2>(cr);
      cg += qperm<kXor2>(cg);
      cb += qperm<kXor2>(cb);
      const float inv_t = tail ? 1.0f / (float)(n - 2) : 0.0f;
      // channel q's plain colour of the selected layers (q = 3: unused)
      const float s1 = q == 0 ? c1.x : (q == 1 ? c1.y : c1.z);
      const float s2 = q == 0 ? c2.x : (q == 1 ? c2.y : c2.z);
      V cq = q == 0 ? cr : (q == 1 ? cg : cb);
      cq -= (V)round_q(s1 * kQ24);
      cq -= (V)round_q(s2 * kQ24);
      const float av = q == 3 ? A * (1.0f / kQ24) : to_f32(cq) * (1.0f / kQ24);
      reinterpret_cast<float*>(a.tail_avg + (j3 * g.w3 + i3))[q] = av * inv_t;
    }
  }
  uint32_t errf = (q == 0 && n > a.max_n) ? STARNT_DERR_COUNT : 0u;
  errf |= zmax > kOne ? STARNT_DERR_DEPTH : 0u;
  errf |= amax > kOne ? STARNT_DERR_ALPHA : 0u;
  if (errf) atomicOr(a.err, errf);
}

// A block covers 64 pixels of one row (x from the thread, y = blockIdx.y), so
// no lane divides to find its pixel and y-dependent values are
// block-uniform: a row off the pass-3 grid streams depths only.
template <bool HALF, bool AVG>
__global__ __launch_bounds__(256) void features_kernel(FeatArgs a) {
  const int q = threadIdx.x & (kG - 1);
  const int x = (int)(blockIdx.x * (256u / kG) + threadIdx.x / kG);
  const int y = (int)blockIdx.y;
  if (x >= a.W) return;  // whole quads leave together
  const int p = y * a.W + x;
  const Grids g = load_grids(a.sched, a.W, a.H);
  const int i2 = grid_index_of(x, a.W, g.w2), j2 = grid_index_of(y, a.H, g.h2);
  const int j3 = grid_index_of(y, a.H, g.h3);
  const uint32_t b = a.off[p], e = a.off[p + 1];
  if (j3 < 0) {
    pixel<HALF, false, AVG, false>(a, g, p, q, b, e, i2, j2, -1, j3);
    return;
  }
  const int i3 = grid_index_of(x, a.W, g.w3);
  // the 64-bit variant only where the wave holds a list longer than kNarrow
  if (__builtin_amdgcn_ballot_w64(e - b > kNarrow) != 0)
    pixel<HALF, true, AVG, true>(a, g, p, q, b, e, i2, j2, i3, j3);
  else
    pixel<HALF, false, AVG, true>(a, g, p, q, b, e, i2, j2, i3, j3);
}

// Features of a list of pixels (re-rendering of untrusted interpolated
// pixels): entry i of the list is pixel p = list[i] of the frame, and its
// outputs go to slot i of compact arrays, all at full resolution. A quad owns
// one entry; quads stride through the list, whose length is read on the
// device. Entries outside the frame and a length above the capacity are
// flagged, not followed.
template <bool HALF>
__global__ __launch_bounds__(256) void features_list_kernel(FeatArgs a) {
  const uint32_t cap = (uint32_t)a.W;
  const uint32_t given = *a.list_n;
  const uint32_t n = given < cap ? given : cap;
  const int q = threadIdx.x & (kG - 1);
  const uint32_t first = (blockIdx.x * (unsigned)blockDim.x + threadIdx.x) / kG;
  const uint32_t stride = gridDim.x * (unsigned)blockDim.x / kG;
  if (first == 0 && q == 0 && given > cap) atomicOr(a.err, STARNT_DERR_LIST);
  Grids g;
  g.w2 = g.w3 = (int)cap;
  g.h2 = g.h3 = 1;
  for (uint32_t i = first; i < n; i += stride) {
    const uint32_t p = a.list[i];
    if (p >= a.frame_p) {
      if (q == 0) atomicOr(a.err, STARNT_DERR_LIST);
      continue;  // the same p for the whole quad
    }
    const uint32_t b = a.off[p], e = a.off[p + 1];
    if (__builtin_amdgcn_ballot_w64(e - b > kNarrow) != 0)
      pixel<HALF, true, false, true>(a, g, (int)i, q, b, e, (int)i, 0, (int)i, 0);
    else
      pixel<HALF, false, false, true>(a, g, (int)i, q, b, e, (int)i, 0, (int)i, 0);
  }
}

}  // namespace

int launch_features_list(const starnt_frags& f, const uint32_t* list, const uint32_t* list_n,
                         const starnt_feats& o, hipStream_t s) {
  FeatArgs a{};
  a.W = o.width;  // capacity: the compact arrays hold o.width entries
  a.H = 1;
  a.off = f.offsets;
  a.depth = f.depth;
  a.rgba = f.rgba;
  a.prim = f.prim;
  a.max_n = f.max_per_pixel;
  a.sched = nullptr;
  a.d1 = o.d1;
  a.layer1 = reinterpret_cast<float4*>(o.layer1);
  a.count = o.count;
  a.layer2 = reinterpret_cast<float4*>(o.layer2);
  a.tail = reinterpret_cast<float4*>(o.tail);
  a.sel = reinterpret_cast<uint2*>(o.sel);
  a.err = o.err;
  a.tail_avg = nullptr;
  a.list = list;
  a.list_n = list_n;
  a.frame_p = (uint32_t)f.width * (uint32_t)f.height;
  // enough quads to fill the chip; each walks the list with a stride
  const int64_t quads = o.width;
  int64_t blocks = (quads * kG + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  const dim3 block(256), grid((unsigned)blocks);
  if (f.rgba_dtype == STARNT_F16) hipLaunchKernelGGL(features_list_kernel<true>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(features_list_kernel<false>, grid, block, 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_patch features launch");
  return STARNT_OK;
}

int launch_features(const starnt_frags& f, const starnt_sched* sched, const starnt_feats& o, hipStream_t s) {
  FeatArgs a{};
  a.W = f.width;
  a.H = f.height;
  a.off = f.offsets;
  a.depth = f.depth;
  a.rgba = f.rgba;
  a.prim = f.prim;
  a.max_n = f.max_per_pixel;
  a.sched = sched;
  a.d1 = o.d1;
  a.layer1 = reinterpret_cast<float4*>(o.layer1);
  a.count = o.count;
  a.layer2 = reinterpret_cast<float4*>(o.layer2);
  a.tail = reinterpret_cast<float4*>(o.tail);
  a.sel = reinterpret_cast<uint2*>(o.sel);
  a.err = o.err;
  const dim3 block(256), grid((unsigned)((f.width + 256 / kG - 1) / (256 / kG)), (unsigned)f.height);
  a.tail_avg = reinterpret_cast<float4*>(o.tail_avg);
  const bool half = f.rgba_dtype == STARNT_F16;
  const LaunchTimer tm = take_launch_timer();
  if (o.tail_avg) {
    if (half) launch_maybe_timed(tm, features_kernel<true, true>, grid, block, s, a);
    else launch_maybe_timed(tm, features_kernel<false, true>, grid, block, s, a);
  } else {
    if (half) launch_maybe_timed(tm, features_kernel<true, false>, grid, block, s, a);
    else launch_maybe_timed(tm, features_kernel<false, false>, grid, block, s, a);
  }
  STARNT_LAUNCH_CHECK("starnt_features launch");
  return STARNT_OK;
}

}  // namespace starnt
