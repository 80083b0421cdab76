// Exact A-buffer composite: every pixel's fragments in (depth, prim) order,
// blended front to back with the over operator (eq (1) with premultiplied
// colour a*c), plus the exact tail colour (sorted positions 3..N alone).
// This is the ground truth the learned path is judged against, the source of
// training targets, and the baseline it must beat on time.
//
// Main kernel: one wave owns PIX consecutive pixels and works alone (a block
// is one wave, so no wave waits on another). It takes its pixels in batches
// of whole lists holding at most CAP fragments (16 pixels; CAP 192, 256 or
// 384, the smallest that holds the declared maximum list length):
//   1. the batch's fragments are loaded with one lane per fragment (every
//      load instruction covers a contiguous run of the CSR arrays); depths
//      and RGBA go to LDS in CSR order;
//   2. each lane ranks its fragments within their list by counting the
//      smaller depths there (depth bits compare as unsigned integers, which
//      orders valid depths in [0, 1] as numbers), eight per LDS round trip:
//      in LDS every list is followed by seven guard keys larger than any
//      depth, so whole 8-key blocks are counted with no mask. Each
//      fragment finds its list's range with no search: every list writes
//      its descriptor (index, start, end) at its first slot, the other slots
//      hold 0, and a prefix maximum over the batch's slots (descriptors grow
//      with the list index) carries each list's descriptor over its slots;
//   3. each fragment writes its index at its sorted slot and reads it back: a
//      slot claimed twice means equal depths in a list, and only then are
//      the ranks recounted on (depth, primitive id) for that batch, with the
//      primitive ids read for that batch alone; the claims are the sorted
//      order (RGBA stays in LDS in CSR order, nothing is moved);
//   4. the walk is split over the lanes: each lane composites CAP / 64
//      consecutive sorted slots, closing a partial composite at every list
//      start, and each pixel lane joins its list's partials in order (the
//      over operator is associative: (C, T) then (C', T') is
//      (C + T C', T T')).
// Inside a batch the transmittance is a plain FP32 product (at most CAP
// factors, relative error below 2^-15); the long-list kernel keeps a
// compensated FP32 product (value + error term).
// Lists longer than CAP are left to a block-wide kernel (launched only when
// the declared maximum list length allows them), which stages up to kCapL
// fragments of a 256-pixel window in LDS.
#include "internal.h"

namespace starnt {
namespace {

// Main-kernel configurations: a wave owns PIX consecutive pixels and takes
// batches of at most CAP fragments. The launch takes the smallest CAP that
// holds the declared maximum list length: small batches keep LDS and
// registers low (more waves per CU hide more latency), larger ones keep
// longer lists out of the much slower long-list kernel. Measured per frame
// when the configurations were chosen (the kernel has since become faster):
// 1080p (mean 8, max 64) 126 us at <192, 16> against 142 us at <192, 32>;
// 4K (mean 16, max 256) 1.71 ms at <256, 16>, 1.98 ms at <384, 16> and 3.4
// ms at <384, 48>; 16-pixel waves were also faster than 8, 12, 20 or 24.
template <int CAP, int PIX>
struct WaveCfg {
  static constexpr int kCap = CAP;
  static constexpr int kPix = PIX;
  static constexpr int kSlots = CAP / 64;  // fragments per lane in a batch
  // keys, seven guards per list and slack; the walk's partials (64 chunks
  // and PIX lists, four words each) reuse the same words
  static constexpr int kKeys = (CAP + 7 * PIX + 8) > 4 * (64 + PIX) ? (CAP + 7 * PIX + 8) : 4 * (64 + PIX);
  static_assert(CAP % 64 == 0 && CAP <= 512 && PIX <= 64, "batch words hold 9-bit indices, 6-bit lists");
};
using CfgSmall = WaveCfg<192, 16>;  // lists up to 192 fragments
using CfgMid = WaveCfg<256, 16>;    // up to 256
using CfgLarge = WaveCfg<384, 16>;  // up to 384 (longer ones: the long-list kernel)
constexpr int kWPB = 1;             // waves per block (each works alone; 2 or 4 measured slower)
constexpr int kPB = 256;     // pixels per window (long-list kernel)
constexpr int kCapL = 2048;  // fragments per LDS batch (long-list kernel)
constexpr uint32_t kOneBits = 0x3F800000u;  // bits of 1.0f

struct ExactArgs {
  int W, H;
  const uint32_t* off;
  const float* depth;
  const void* rgba;
  const uint32_t* prim;
  uint32_t max_n;
  float bg0, bg1, bg2;
  float* rgb;
  float* fstar;
  uint32_t* err;
};

// T <- T * (1 - a) with T kept as th + tl (double-float)
__device__ __forceinline__ void trans_mul(float& th, float& tl, float a) {
  const float mh = 1.0f - a;
  const float ml = -a - (mh - 1.0f);      // exact error of 1 - a (|1| >= |a|)
  const float p = th * mh;
  const float pe = fmaf(th, mh, -p);      // exact error of th * mh
  const float lo = pe + fmaf(th, ml, tl * mh);
  const float s = p + lo;
  tl = lo - (s - p);
  th = s;
}

// Front-to-back state of one pixel: colour C, transmittance T = th + tl, and
// the tail alone (sorted positions 3..N) F with its transmittance uh + ul.
struct Walk {
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, th = 1.0f, tl = 0.0f;
  float F0 = 0.f, F1 = 0.f, F2 = 0.f, uh = 1.0f, ul = 0.0f;
};

template <bool FSTAR>
__device__ __forceinline__ void walk_step(Walk& w, float4 c, bool tail) {
  const float al = fminf(fmaxf(c.w, 0.0f), 1.0f);
  const float t = w.th + w.tl;
  w.C0 = fmaf(t * al, c.x, w.C0);
  w.C1 = fmaf(t * al, c.y, w.C1);
  w.C2 = fmaf(t * al, c.z, w.C2);
  trans_mul(w.th, w.tl, al);
  if (FSTAR && tail) {
    const float u = w.uh + w.ul;
    w.F0 = fmaf(u * al, c.x, w.F0);
    w.F1 = fmaf(u * al, c.y, w.F1);
    w.F2 = fmaf(u * al, c.z, w.F2);
    trans_mul(w.uh, w.ul, al);
  }
}

__device__ __forceinline__ void write_pixel(const ExactArgs& a, int p, const Walk& w) {
  const float T = w.th + w.tl;
  a.rgb[3 * (size_t)p + 0] = fmaf(T, a.bg0, w.C0);
  a.rgb[3 * (size_t)p + 1] = fmaf(T, a.bg1, w.C1);
  a.rgb[3 * (size_t)p + 2] = fmaf(T, a.bg2, w.C2);
  if (a.fstar) {
    a.fstar[3 * (size_t)p + 0] = w.F0;
    a.fstar[3 * (size_t)p + 1] = w.F1;
    a.fstar[3 * (size_t)p + 2] = w.F2;
  }
}

// Inclusive prefix maximum over the 64 lanes of a wave, in lane order: a
// Hillis-Steele scan inside each 16-lane row (row_shr 1, 2, 4, 8; lanes
// shifted in from outside the row read 0), then the last lane of row 0 into
// row 1 and of row 2 into row 3 (row_bcast:15), then lane 31 into rows 2 and
// 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_max_scan(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
  return v;
}

// LDS written by some lanes of a wave and read by others: the wave's own
// ordering point (waves of a block never share data)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Composite of a run of sorted slots (over operator, plain FP32: the
// transmittance of at most 384 factors stays within 2^-15 relative)
struct Part {
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.0f;
  __device__ __forceinline__ void add(float4 c) {
    const float al = fminf(fmaxf(c.w, 0.0f), 1.0f);
    const float ta = T * al;
    C0 = fmaf(ta, c.x, C0);
    C1 = fmaf(ta, c.y, C1);
    C2 = fmaf(ta, c.z, C2);
    T = fmaf(-T, al, T);
  }
  __device__ __forceinline__ float4 get() const { return make_float4(C0, C1, C2, T); }
};

// Slot-claim word: the fragment index in bits 0-8, and at a list's first
// sorted slot the list's index in the batch in bits 9-14 and bit 15 set
constexpr uint32_t kIdxMask = 0x1FFu;
constexpr uint32_t kStartBit = 0x8000u;

// A fragment's list descriptor in a batch, (list << 20) | (start << 10) |
// end, kept in one register per fragment and unpacked where used
__device__ __forceinline__ int desc_start(uint32_t d) { return (int)((d >> 10) & 0x3FFu); }
__device__ __forceinline__ int desc_end(uint32_t d) { return (int)(d & 0x3FFu); }
// the list's shift in the key words: seven guards after every earlier list
__device__ __forceinline__ int desc_shift(uint32_t d) { return 7 * (int)(d >> 20); }
// the claim word's list-start bits, for the fragment that sorts first
__device__ __forceinline__ uint32_t desc_first(uint32_t d) { return kStartBit | ((d >> 20) << 9); }

// Chunked walk of a batch's sorted slots: lane l composites slots
// [kSlots l, kSlots l + kSlots), closing a segment at every list start. A
// chunk's segment before its first list start (the whole chunk if none
// starts in it) goes to s_part[l]; the segment from a list's start to its
// end or the chunk's end goes to s_part[64 + list]. TAIL leaves out each
// list's first two slots (the tail colour).
template <int kSlots, bool TAIL>
__device__ __forceinline__ void chunk_walk(const float4* s_c, const uint16_t* s_idx, float4* s_part, int l, int m) {
  Part pt;
  int open = -1;
  const int t0 = kSlots * l;
  // TAIL: whether the slot before the chunk starts a list (then the chunk's
  // first slot is its list's second)
  bool prev_start = TAIL && t0 > 0 && t0 < m && (s_idx[t0 - 1] & kStartBit);
#pragma unroll
  for (int u = 0; u < kSlots; ++u) {
    const int t = t0 + u;
    if (t < m) {
      const uint32_t q = s_idx[t];
      const bool st = (q & kStartBit) != 0;
      if (st) {
        s_part[open < 0 ? l : 64 + open] = pt.get();
        pt = Part();
        open = (int)((q >> 9) & 63u);
      }
      if (!TAIL || !(st || prev_start)) pt.add(s_c[q & kIdxMask]);
      prev_start = st;
    }
  }
  s_part[open < 0 ? l : 64 + open] = pt.get();
}

// A list's composite from the chunk partials: its own segment, then the
// head segment of every later chunk it reaches
template <int kSlots>
__device__ __forceinline__ float4 list_result(const float4* s_part, int lid, int s0, int n) {
  float4 r = s_part[64 + lid];
  const int q2 = (s0 + n - 1) / kSlots;
  for (int q = s0 / kSlots + 1; q <= q2; ++q) {
    const float4 h = s_part[q];
    r.x = fmaf(r.w, h.x, r.x);
    r.y = fmaf(r.w, h.y, r.y);
    r.z = fmaf(r.w, h.z, r.z);
    r.w *= h.w;
  }
  return r;
}

// Waves per SIMD asked of the register allocator: the 192-fragment colour
// kernel fits 64 registers without spilling, so 8 waves per SIMD (LDS allows
// 33 waves per CU); 1080p 125.1 against 126.5 us at 7 waves, 1440p 720
// against 734 us. The tail variant and larger batches keep their registers
// (a cap spills there, and LDS caps their waves anyway).
template <class Cfg, bool FSTAR>
constexpr int exact_waves_per_simd() { return (Cfg::kCap == 192 && !FSTAR) ? 8 : 1; }

template <class Cfg, bool HALF, bool FSTAR>
__global__ __launch_bounds__(64 * kWPB) __attribute__((amdgpu_waves_per_eu(exact_waves_per_simd<Cfg, FSTAR>())))
void exact_wave_kernel(ExactArgs a) {
  constexpr int kCapW = Cfg::kCap;
  constexpr int kSlots = Cfg::kSlots;
  constexpr int kKeys = Cfg::kKeys;
  // s_key: first each list's descriptor, (list << 20) | (start << 10) | end,
  // at the list's first slot (0 elsewhere); then the depth bits of list L's
  // fragments at positions start + 7 L, so every list is followed by seven keys larger than any
  // depth (the batch holds at most 64 lists): a count over whole 8-key
  // blocks from a list's start reads no other list's keys and needs no mask.
  // After the ranking it holds the chunk partials of the walk.
  __shared__ __align__(16) uint32_t s_key_all[kWPB][kKeys];
  __shared__ float4 s_c_all[kWPB][kCapW];        // RGBA in CSR order (prim ids in a recount)
  __shared__ uint16_t s_idx_all[kWPB][kCapW];    // slot claims: the sorted order
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // one value per wave
  uint32_t* s_key = s_key_all[wv];
  float4* s_c = s_c_all[wv];
  uint16_t* s_idx = s_idx_all[wv];
  float4* s_part = reinterpret_cast<float4*>(s_key);   // [64 + PIX] chunk and list partials

  const int l = (int)(threadIdx.x & 63);
  const int P = a.W * a.H;
  const int p0 = ((int)blockIdx.x * kWPB + wv) * Cfg::kPix;
  if (p0 >= P) return;  // a whole wave past the frame
  const int np = min(Cfg::kPix, P - p0);
  const int p = p0 + l;
  const bool valid = l < np;
  const uint32_t b = a.off[valid ? p : P];
  const uint32_t e = a.off[valid ? p + 1 : P];
  const uint32_t n = e - b;
  uint32_t errf = (valid && n > a.max_n) ? STARNT_DERR_COUNT : 0u;
  const bool lng = valid && n > (uint32_t)kCapW;  // left to the long-list kernel
  const uint64_t longmask = __builtin_amdgcn_ballot_w64(lng);
  Walk w;

  int cur = 0;
  while (cur < np) {
    if ((longmask >> cur) & 1ull) {
      ++cur;
      continue;
    }
    // the batch: lanes cur .. end-1, whole lists, at most kCapW fragments,
    // no long list inside (ends are increasing, so the fitting lanes form a
    // prefix; lane cur always fits)
    const uint32_t bcur = (uint32_t)__builtin_amdgcn_readlane((int)b, cur);
    const bool fit = valid && l >= cur && e - bcur <= (uint32_t)kCapW;
    const uint64_t stop = ~(__builtin_amdgcn_ballot_w64(fit) >> cur) | (longmask >> cur);
    const int cnt = min(stop ? (int)__builtin_ctzll(stop) : 64 - cur, np - cur);
    const int end = cur + cnt;
    const int m = (int)((uint32_t)__builtin_amdgcn_readlane((int)e, end - 1) - bcur);
    const bool mine = l >= cur && l < end;
    const int s0 = (int)(b - bcur);  // this lane's list in the batch (when mine)
    if (m > 0) {
      // 1. loads: clamped indices keep every load in the batch, so all of
      // them are issued before the first use
      uint32_t zb[kSlots];
      float4 c[kSlots];
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        const int i = min(l + 64 * k, m - 1);
        zb[k] = __float_as_uint(a.depth[bcur + i]);
        c[k] = load_rgba<HALF>(a.rgba, bcur + i);
      }
      // each nonempty list's descriptor at its first slot, 0 at the others
      // (in the key words, read before any key is written; a wave's LDS
      // writes land in program order); RGBA goes to LDS in CSR order as it
      // arrives (lanes past the batch repeat its last fragment, the same
      // value to the same place)
#pragma unroll
      for (int k = 0; k < kSlots; ++k)
        if (l + 64 * k < m) s_key[l + 64 * k] = 0u;
      if (mine && n > 0)
        s_key[s0] = ((uint32_t)(l - cur) << 20) | ((uint32_t)s0 << 10) | (uint32_t)(s0 + (int)n);
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        errf |= (l + 64 * k < m && !(c[k].w >= 0.0f && c[k].w <= 1.0f)) ? STARNT_DERR_ALPHA : 0u;
        s_c[min(l + 64 * k, m - 1)] = c[k];
      }
      wave_sync();
      int pos[kSlots];
      uint32_t dd[kSlots];
      // each fragment's descriptor: the prefix maximum up to its slot, in
      // blocks of 64 slots (run: the maximum over the earlier blocks)
      uint32_t run = 0;
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        const int i = l + 64 * k;
        pos[k] = 0;
        dd[k] = max(wave_max_scan(i < m ? s_key[i] : 0u), run);
        run = (uint32_t)__builtin_amdgcn_readlane((int)dd[k], 63);
        if (i < m) errf |= zb[k] > kOneBits ? STARNT_DERR_DEPTH : 0u;  // negatives, -0 and NaN too
      }
      wave_sync();  // descriptors read before keys overwrite them
      // keys, and the seven guard keys after every list
#pragma unroll
      for (int k = 0; k < kSlots; ++k)
        if (l + 64 * k < m) s_key[l + 64 * k + desc_shift(dd[k])] = zb[k];
      if (mine) {
#pragma unroll
        for (int g = 0; g < 7; ++g) s_key[s0 + (int)n + 7 * (l - cur) + g] = 0xFFFFFFFFu;
      }
      wave_sync();  // keys written
      // 2. ranks: the count of smaller depths from the list's start, eight
      // per LDS round trip (depth bits compare as unsigned integers, which
      // orders valid depths in [0, 1] as numbers)
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        const int i = l + 64 * k;
        if (i < m) {
          int r = 0;
          const uint32_t zi = min(zb[k], kOneBits);  // out-of-range depths (flagged) below the guards
          const int sh = desc_shift(dd[k]);
          for (int j = desc_start(dd[k]) + sh; j < desc_end(dd[k]) + sh; j += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = s_key[j + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) r += v[u] < zi ? 1 : 0;
          }
          pos[k] = desc_start(dd[k]) + r;
          s_idx[pos[k]] = (uint16_t)(i | (r == 0 ? desc_first(dd[k]) : 0u));
        }
      }
      wave_sync();
      // 3. every slot claimed once, or equal depths somewhere in the batch:
      // then exact ranks on (depth, prim), and the claims written again
      bool clash = false;
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        const int i = l + 64 * k;
        if (i < m) clash |= (s_idx[pos[k]] & kIdxMask) != (uint32_t)i;
      }
      if (__builtin_amdgcn_ballot_w64(clash)) {
        // prim ids beside the colours: s_c holds kCapW float4, the ids take
        // the words after the first kCapW
        uint32_t* s_pr = reinterpret_cast<uint32_t*>(s_c) + 3 * kCapW;
        uint32_t pr[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
          const int i = l + 64 * k;
          pr[k] = 0;
          if (i < m) {
            pr[k] = a.prim[bcur + i];
            s_pr[i] = pr[k];
          }
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
          const int i = l + 64 * k;
          if (i < m) {
            // the full key (depth, prim); equal keys (outside the input
            // contract) keep their staging order, so the ranks always form a
            // permutation of the list's slots
            int r = 0;
            const int sh = desc_shift(dd[k]);
            for (int j = desc_start(dd[k]); j < desc_end(dd[k]); ++j) {
              const uint32_t zj = s_key[j + sh], pj = s_pr[j];
              r += (zj < zb[k]) | ((zj == zb[k]) & ((pj < pr[k]) | ((pj == pr[k]) & (j < i))));
            }
            pos[k] = desc_start(dd[k]) + r;
          }
        }
        wave_sync();  // keys and prim ids read before the colours are restored
        // the colours the prim ids displaced, read again (this rare path
        // waits on each reload rather than holding them all in registers)
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
          const int i = l + 64 * k;
          s_c[min(i, m - 1)] = load_rgba<HALF>(a.rgba, bcur + min(i, m - 1));
          if (i < m) s_idx[pos[k]] = (uint16_t)(i | (pos[k] == desc_start(dd[k]) ? desc_first(dd[k]) : 0u));
        }
      }
      wave_sync();  // claims final, keys no longer read
      // 4. the walk: chunk partials, then each pixel lane combines its list's
      chunk_walk<kSlots, false>(s_c, s_idx, s_part, l, m);
      wave_sync();
      if (mine && n > 0) {
        const float4 r = list_result<kSlots>(s_part, l - cur, s0, (int)n);
        w.C0 = r.x;
        w.C1 = r.y;
        w.C2 = r.z;
        w.th = r.w;
      }
      if (FSTAR) {
        wave_sync();  // colour partials read before the tail's overwrite them
        chunk_walk<kSlots, true>(s_c, s_idx, s_part, l, m);
        wave_sync();
        if (mine && n > 0) {
          const float4 r = list_result<kSlots>(s_part, l - cur, s0, (int)n);
          w.F0 = r.x;
          w.F1 = r.y;
          w.F2 = r.z;
        }
      }
      wave_sync();  // the next batch reuses the LDS arrays
    }
    cur = end;
  }
  // a long list is the long-list kernel's, unless the declared maximum ruled
  // that kernel out: then the list broke the declaration (flagged above) and
  // the pixel gets the background alone, so every output is defined
  if (valid && (!lng || a.max_n <= (uint32_t)kCapW)) write_pixel(a, p, w);
  if (errf && a.err) atomicOr(a.err, errf);
}

// Lists longer than kCapW (up to kCapL): a block owns a window of 256 pixels
// and returns at once unless one of them is long. The window's fragments are
// staged in LDS in batches of at most kCapL with coalesced loads, each
// fragment's rank within its list is counted there on the full key, the rank
// scatters it into sorted order, and one thread per long pixel walks its list.
template <int kCapW, bool HALF, bool FSTAR>
__global__ __launch_bounds__(256) void exact_long_kernel(ExactArgs a) {
  __shared__ uint32_t s_off[kPB + 1];
  __shared__ float s_z[kCapL];
  __shared__ uint32_t s_pr[kCapL];
  __shared__ float4 s_c[kCapL];
  __shared__ uint16_t s_ord[kCapL];

  const int P = a.W * a.H;
  const int p0 = blockIdx.x * kPB;
  const int npix = min(kPB, P - p0);
  const int tid = threadIdx.x;
  const uint32_t n_me = tid < npix ? a.off[p0 + tid + 1] - a.off[p0 + tid] : 0u;
  const bool lng = n_me > (uint32_t)kCapW;
  if (!__syncthreads_or(lng)) return;
  for (int i = tid; i <= npix; i += blockDim.x) s_off[i] = a.off[p0 + i];
  __syncthreads();

  uint32_t errf = (lng && n_me > a.max_n) ? STARNT_DERR_COUNT : 0u;
  Walk w;
  int bs = 0;
  while (bs < npix) {
    const uint32_t fs = s_off[bs];
    // largest be in (bs, npix] with s_off[be] - fs <= kCapL
    int lo = bs + 1, hi = npix;
    if (s_off[lo] - fs > (uint32_t)kCapL) {
      hi = lo;  // a single list longer than kCapL: rejected on the host
    } else {
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] - fs <= (uint32_t)kCapL) lo = mid; else hi = mid - 1;
      }
    }
    const int be = lo;
    const int cnt = (int)min(s_off[be] - fs, (uint32_t)kCapL);
    for (int i = tid; i < cnt; i += blockDim.x) {
      const float z = a.depth[fs + i];
      const float4 c = load_rgba<HALF>(a.rgba, fs + i);
      s_z[i] = z;
      s_pr[i] = a.prim[fs + i];
      s_c[i] = c;
    }
    __syncthreads();
    for (int i = tid; i < cnt; i += blockDim.x) {
      // list of fragment i: last q in [bs, be) with s_off[q] - fs <= i
      int ql = bs, qh = be - 1;
      while (ql < qh) {
        const int mid = (ql + qh + 1) >> 1;
        if ((int)(s_off[mid] - fs) <= i) ql = mid; else qh = mid - 1;
      }
      const int sb = (int)(s_off[ql] - fs), se = min((int)(s_off[ql + 1] - fs), cnt);
      if (se - sb <= kCapW) continue;  // short lists belong to the main kernel
      const uint32_t zi = __float_as_uint(s_z[i]), pi = s_pr[i];
      int r = 0;
      for (int j = sb; j < se; ++j) {
        const uint32_t zj = __float_as_uint(s_z[j]), pj = s_pr[j];
        r += (zj < zi) | ((zj == zi) & ((pj < pi) | ((pj == pi) & (j < i))));
      }
      s_ord[sb + r] = (uint16_t)i;
      errf |= zi > kOneBits ? STARNT_DERR_DEPTH : 0u;
      errf |= (s_c[i].w >= 0.0f && s_c[i].w <= 1.0f) ? 0u : STARNT_DERR_ALPHA;
    }
    __syncthreads();
    if (lng && tid >= bs && tid < be) {
      const int sb = (int)(s_off[tid] - fs), se = min((int)(s_off[tid + 1] - fs), cnt);
      for (int r = sb; r < se; ++r) walk_step<FSTAR>(w, s_c[s_ord[r]], r - sb >= 2);
    }
    __syncthreads();
    bs = be;
  }
  if (lng) write_pixel(a, p0 + tid, w);
  if (errf && a.err) atomicOr(a.err, errf);
}

template <class Cfg, bool HALF, bool FSTAR>
void launch_exact_c(const ExactArgs& a, uint32_t max_n, hipStream_t s) {
  const int P = a.W * a.H;
  const int waves = (P + Cfg::kPix - 1) / Cfg::kPix;
  launch_maybe_timed(take_launch_timer(), exact_wave_kernel<Cfg, HALF, FSTAR>, dim3((waves + kWPB - 1) / kWPB),
                     dim3(64 * kWPB), s, a);
  // the long-list kernel only where the declared maximum allows such lists
  // (only the largest configuration leaves any)
  if constexpr (Cfg::kCap == CfgLarge::kCap) {
    if (max_n > (uint32_t)Cfg::kCap)
      hipLaunchKernelGGL((exact_long_kernel<Cfg::kCap, HALF, FSTAR>), dim3((P + kPB - 1) / kPB), dim3(256), 0, s,
                         a);
  }
}

// The smallest configuration whose batches hold every declared list
template <bool HALF, bool FSTAR>
void launch_exact_t(const ExactArgs& a, uint32_t max_n, hipStream_t s) {
  if (max_n <= (uint32_t)CfgSmall::kCap) launch_exact_c<CfgSmall, HALF, FSTAR>(a, max_n, s);
  else if (max_n <= (uint32_t)CfgMid::kCap) launch_exact_c<CfgMid, HALF, FSTAR>(a, max_n, s);
  else launch_exact_c<CfgLarge, HALF, FSTAR>(a, max_n, s);
}

}  // namespace

int launch_exact(const starnt_frags& f, const float bg[3], float* rgb, float* fstar, uint32_t* err,
                 hipStream_t s) {
  if (f.max_per_pixel > (uint32_t)kCapL)
    return fail(STARNT_EUNSUPPORTED, "exact composite: max_per_pixel above 2048 is not supported");
  ExactArgs a;
  a.W = f.width;
  a.H = f.height;
  a.off = f.offsets;
  a.depth = f.depth;
  a.rgba = f.rgba;
  a.prim = f.prim;
  a.max_n = f.max_per_pixel;
  a.bg0 = bg[0];
  a.bg1 = bg[1];
  a.bg2 = bg[2];
  a.rgb = rgb;
  a.fstar = fstar;
  a.err = err;
  const bool half = f.rgba_dtype == STARNT_F16;
  if (half) {
    if (fstar) launch_exact_t<true, true>(a, f.max_per_pixel, s);
    else launch_exact_t<true, false>(a, f.max_per_pixel, s);
  } else {
    if (fstar) launch_exact_t<false, true>(a, f.max_per_pixel, s);
    else launch_exact_t<false, false>(a, f.max_per_pixel, s);
  }
  STARNT_LAUNCH_CHECK("starnt_composite (exact) launch");
  return STARNT_OK;
}

}  // namespace starnt
