// Exact A-buffer composite: every pixel's fragments in (depth, prim) order,
// blended front to back with the over operator (eq (1) with premultiplied
// colour a*c), plus the exact tail colour (sorted positions 3..N alone).
// This is the ground truth the learned path is judged against, the source of
// training targets, and the baseline it must beat on time.
//
// Block layout: 256 threads own a window of 256 consecutive pixels. The
// window's fragments are staged in LDS in batches of at most kCap with
// coalesced loads. Each fragment's rank within its pixel is counted in LDS
// (all lanes of a pixel read the same keys, so reads broadcast), the rank
// scatters it into sorted order, and one thread per pixel walks its sorted
// list. The transmittance is a compensated FP32 product (value + error term).
#include "internal.h"

namespace starnt {
namespace {

constexpr int kPB = 256;     // pixels per window
constexpr int kCap = 2048;   // fragments per LDS batch

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

template <bool HALF>
__global__ __launch_bounds__(256) void exact_kernel(ExactArgs a) {
  __shared__ uint32_t s_off[kPB + 1];
  __shared__ float s_z[kCap];
  __shared__ uint32_t s_pr[kCap];
  __shared__ float4 s_c[kCap];
  __shared__ uint16_t s_ord[kCap];

  const int P = a.W * a.H;
  const int p0 = blockIdx.x * kPB;
  const int npix = min(kPB, P - p0);
  const int tid = threadIdx.x;
  for (int i = tid; i <= npix; i += blockDim.x) s_off[i] = a.off[p0 + i];
  __syncthreads();

  uint32_t errf = 0;
  // per-thread pixel state (thread tid owns pixel p0 + tid)
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, th = 1.0f, tl = 0.0f;
  float F0 = 0.f, F1 = 0.f, F2 = 0.f, uh = 1.0f, ul = 0.0f;
  if (tid < npix) {
    const uint32_t n = s_off[tid + 1] - s_off[tid];
    if (n > a.max_n) errf |= STARNT_DERR_COUNT;
  }

  int bs = 0;
  while (bs < npix) {
    const uint32_t fs = s_off[bs];
    // largest be in (bs, npix] with s_off[be] - fs <= kCap
    int lo = bs + 1, hi = npix;
    if (s_off[lo] - fs > (uint32_t)kCap) {
      hi = lo;  // a single list longer than kCap: rejected on the host
    } else {
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] - fs <= (uint32_t)kCap) lo = mid; else hi = mid - 1;
      }
    }
    const int be = lo;
    const int cnt = (int)min(s_off[be] - fs, (uint32_t)kCap);
    for (int i = tid; i < cnt; i += blockDim.x) {
      const float z = a.depth[fs + i];
      const float4 c = load_rgba<HALF>(a.rgba, fs + i);
      errf |= (z >= 0.0f && z <= 1.0f) ? 0u : STARNT_DERR_DEPTH;
      errf |= (c.w >= 0.0f && c.w <= 1.0f) ? 0u : STARNT_DERR_ALPHA;
      s_z[i] = z;
      s_pr[i] = a.prim[fs + i];
      s_c[i] = c;
    }
    __syncthreads();
    // rank of each fragment within its pixel
    for (int i = tid; i < cnt; i += blockDim.x) {
      // pixel q of fragment i: last q in [bs, be) with s_off[q] - fs <= i
      int ql = bs, qh = be - 1;
      while (ql < qh) {
        const int mid = (ql + qh + 1) >> 1;
        if ((int)(s_off[mid] - fs) <= i) ql = mid; else qh = mid - 1;
      }
      const int sb = (int)(s_off[ql] - fs), se = min((int)(s_off[ql + 1] - fs), cnt);
      const float zi = s_z[i];
      const uint32_t pi = s_pr[i];
      int r = 0;
      // ties of the whole key (not allowed by the input contract) fall back to
      // staging order so the ranks always form a permutation
      for (int j = sb; j < se; ++j) {
        const float zj = s_z[j];
        const uint32_t pj = s_pr[j];
        r += (zj < zi) | ((zj == zi) & ((pj < pi) | ((pj == pi) & (j < i))));
      }
      s_ord[sb + r] = (uint16_t)i;
    }
    __syncthreads();
    if (tid >= bs && tid < be) {
      const int sb = (int)(s_off[tid] - fs), se = min((int)(s_off[tid + 1] - fs), cnt);
      for (int r = sb; r < se; ++r) {
        const float4 c = s_c[s_ord[r]];
        const float al = fminf(fmaxf(c.w, 0.0f), 1.0f);
        const float t = th + tl;
        C0 = fmaf(t * al, c.x, C0);
        C1 = fmaf(t * al, c.y, C1);
        C2 = fmaf(t * al, c.z, C2);
        trans_mul(th, tl, al);
        if (r - sb >= 2) {
          const float u = uh + ul;
          F0 = fmaf(u * al, c.x, F0);
          F1 = fmaf(u * al, c.y, F1);
          F2 = fmaf(u * al, c.z, F2);
          trans_mul(uh, ul, al);
        }
      }
    }
    __syncthreads();
    bs = be;
  }
  if (tid < npix) {
    const int p = p0 + tid;
    const float T = th + tl;
    a.rgb[3 * (size_t)p + 0] = fmaf(T, a.bg0, C0);
    a.rgb[3 * (size_t)p + 1] = fmaf(T, a.bg1, C1);
    a.rgb[3 * (size_t)p + 2] = fmaf(T, a.bg2, C2);
    if (a.fstar) {
      a.fstar[3 * (size_t)p + 0] = F0;
      a.fstar[3 * (size_t)p + 1] = F1;
      a.fstar[3 * (size_t)p + 2] = F2;
    }
  }
  if (errf && a.err) atomicOr(a.err, errf);
}

}  // namespace

int launch_exact(const starnt_frags& f, const float bg[3], float* rgb, float* fstar, uint32_t* err,
                 hipStream_t s) {
  if (f.max_per_pixel > (uint32_t)kCap)
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
  const int P = f.width * f.height;
  const dim3 block(256), grid((P + kPB - 1) / kPB);
  if (f.rgba_dtype == STARNT_F16)
    hipLaunchKernelGGL(exact_kernel<true>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(exact_kernel<false>, grid, block, 0, s, a);
  STARNT_LAUNCH_CHECK("starnt_composite (exact) launch");
  return STARNT_OK;
}

}  // namespace starnt
