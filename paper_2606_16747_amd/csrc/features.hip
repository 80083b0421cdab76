// Passes 1-3 of STAR-NT (Sec. 3, Fig. 1) over per-pixel fragment lists.
//
// One thread owns one pixel and streams its list once:
//  * pass 1 (every pixel): nearest fragment by (depth, prim) -> d1, layer 1, N;
//  * pass 2 (pixels sampled by the pass-2 grid): second-nearest -> layer 2;
//  * pass 3 (pixels sampled by the pass-3 grid): order-independent sums over
//    ALL fragments in exact fixed point, then the two selected layers are
//    subtracted exactly, leaving the tail (sorted positions 3..N):
//      A = sum a (Q31), S = sum a c (Q31, a c rounded once in FP32),
//      Lg = sum -log2(1 - a) (Q27), a = 1 counted apart (zero transmittance),
//    giving x = (N, t_tail = 2^-Lg, Ct = S / A) (Sec. 3.3).
// Integer sums make every output independent of the order of a list.
#include "internal.h"

namespace starnt {
namespace {

constexpr float kQ31 = 2147483648.0f;   // 2^31
constexpr float kQ27 = 134217728.0f;    // 2^27
constexpr uint32_t kNone = 0xFFFFFFFFu;

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
};

// fixed-point quantisers: round to nearest even, exact integers
__device__ __forceinline__ uint32_t q31(float v) { return (uint32_t)__builtin_rintf(v * kQ31); }
__device__ __forceinline__ uint32_t q27(float v) { return (uint32_t)__builtin_rintf(v * kQ27); }

struct FragQ {
  uint32_t a, r, g, b, lg;
  uint32_t opaque;
};

// the per-fragment terms of the tail sums (identical code for the stream and
// for the exact subtraction of the two selected layers)
__device__ __forceinline__ FragQ frag_terms(float4 c) {
  FragQ q;
  float a = fminf(fmaxf(c.w, 0.0f), 1.0f);
  q.a = q31(a);
  q.r = q31(a * c.x);
  q.g = q31(a * c.y);
  q.b = q31(a * c.z);
  if (a >= 1.0f) {
    q.opaque = 1;
    q.lg = 0;
  } else {
    q.opaque = 0;
    q.lg = q27(-__log2f(1.0f - a));
  }
  return q;
}

// (z, prim) order with lazy primitive reads: prim is loaded only on equal depth
__device__ __forceinline__ bool key_less(float z, uint32_t k, float zb, uint32_t kb, const uint32_t* prim) {
  if (z < zb) return true;
  if (z > zb || kb == kNone) return false;
  if (z != zb) return false;  // NaN
  return prim[k] < prim[kb];
}

template <bool HALF>
__global__ __launch_bounds__(256) void features_kernel(FeatArgs a) {
  const int P = a.W * a.H;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const Grids g = load_grids(a.sched, a.W, a.H);
  const int x = p % a.W, y = p / a.W;
  const int i2 = grid_index_of(x, a.W, g.w2), j2 = grid_index_of(y, a.H, g.h2);
  const int i3 = grid_index_of(x, a.W, g.w3), j3 = grid_index_of(y, a.H, g.h3);
  const bool pass2 = (i2 >= 0) & (j2 >= 0);
  const bool pass3 = (i3 >= 0) & (j3 >= 0);

  const uint32_t b = a.off[p], e = a.off[p + 1];
  const uint32_t n = e - b;
  uint32_t errf = n > a.max_n ? STARNT_DERR_COUNT : 0u;

  float z1 = __builtin_inff(), z2 = __builtin_inff();
  uint32_t k1 = kNone, k2 = kNone;
  float4 c1 = make_float4(0.f, 0.f, 0.f, 0.f), c2 = c1;
  uint64_t sa = 0, sr = 0, sg = 0, sb = 0, sl = 0;
  uint32_t nop = 0;

  if (pass3) {
    for (uint32_t k = b; k < e; ++k) {
      const float z = a.depth[k];
      const float4 c = load_rgba<HALF>(a.rgba, k);
      errf |= (z >= 0.0f && z <= 1.0f) ? 0u : STARNT_DERR_DEPTH;
      errf |= (c.w >= 0.0f && c.w <= 1.0f) ? 0u : STARNT_DERR_ALPHA;
      const FragQ q = frag_terms(c);
      sa += q.a; sr += q.r; sg += q.g; sb += q.b; sl += q.lg; nop += q.opaque;
      if (key_less(z, k, z1, k1, a.prim)) {
        z2 = z1; k2 = k1; c2 = c1;
        z1 = z; k1 = k; c1 = c;
      } else if (key_less(z, k, z2, k2, a.prim)) {
        z2 = z; k2 = k; c2 = c;
      }
    }
  } else {
    for (uint32_t k = b; k < e; ++k) {
      const float z = a.depth[k];
      errf |= (z >= 0.0f && z <= 1.0f) ? 0u : STARNT_DERR_DEPTH;
      if (key_less(z, k, z1, k1, a.prim)) {
        z2 = z1; k2 = k1;
        z1 = z; k1 = k;
      } else if (key_less(z, k, z2, k2, a.prim)) {
        z2 = z; k2 = k;
      }
    }
    if (k1 != kNone) c1 = load_rgba<HALF>(a.rgba, k1);
    if (pass2 && k2 != kNone) c2 = load_rgba<HALF>(a.rgba, k2);
  }
  const float a1 = fminf(fmaxf(c1.w, 0.0f), 1.0f);
  const float a2 = fminf(fmaxf(c2.w, 0.0f), 1.0f);

  a.d1[p] = n ? z1 : 1.0f;
  a.layer1[p] = make_float4(a1 * c1.x, a1 * c1.y, a1 * c1.z, a1);
  a.count[p] = n;
  if (a.sel) a.sel[p] = make_uint2(k1, k2);
  if (pass2) a.layer2[(size_t)j2 * g.w2 + i2] = make_float4(a2 * c2.x, a2 * c2.y, a2 * c2.z, a2);
  if (pass3) {
    if (k1 != kNone) {
      const FragQ q = frag_terms(c1);
      sa -= q.a; sr -= q.r; sg -= q.g; sb -= q.b; sl -= q.lg; nop -= q.opaque;
    }
    if (k2 != kNone) {
      const FragQ q = frag_terms(c2);
      sa -= q.a; sr -= q.r; sg -= q.g; sb -= q.b; sl -= q.lg; nop -= q.opaque;
    }
    float tt = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f, A = 0.f;
    if (n > 2) {
      tt = nop ? 0.0f : exp2f(-(float)sl * (1.0f / kQ27));
      if (sa) {
        const float inv = 1.0f / (float)sa;
        cr = (float)sr * inv;
        cg = (float)sg * inv;
        cb = (float)sb * inv;
      }
      A = (float)sa * (1.0f / kQ31);
    }
    float4* t = a.tail + 2 * ((size_t)j3 * g.w3 + i3);
    t[0] = make_float4((float)n, tt, cr, cg);
    t[1] = make_float4(cb, A, 0.0f, 0.0f);
  }
  if (errf) atomicOr(a.err, errf);
}

}  // namespace

int launch_features(const starnt_frags& f, const starnt_sched* sched, const starnt_feats& o, hipStream_t s) {
  FeatArgs a;
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
  const int P = f.width * f.height;
  const dim3 block(256), grid((P + 255) / 256);
  if (f.rgba_dtype == STARNT_F16)
    hipLaunchKernelGGL(features_kernel<true>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(features_kernel<false>, grid, block, 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_features launch");
  return STARNT_OK;
}

}  // namespace starnt
