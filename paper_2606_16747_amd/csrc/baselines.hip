// Cheap approximate baselines of the evaluation (Sec. 4), on the same
// fragment lists as the method:
//  * weighted blended OIT (McGuire and Bavoil 2013) with the weight driven by
//    window-space depth, w(z, a) = a max(1e-2, 3e3 (1 - z)^3):
//      C = (sum w a c / sum w a) (1 - R) + R C_b,  R = prod (1 - a);
//  * blending in stored (primitive) order with no sort: eq (1) applied to the
//    list as it is, the naive renderer whose error is the paper's E_random.
//
// Layout as in the fragment pass: four lanes own a pixel and stride through
// its list together, so each load instruction of a quad covers a contiguous
// run of the CSR arrays. WBOIT sums are order free and are merged across the
// quad at the end. Over is associative but not commutative: each group of
// four consecutive fragments (one per lane) is combined in list order with
// two in-quad scan steps, then appended to the running (colour,
// transmittance) state, which every lane of the quad holds.
#include "internal.h"

namespace starnt {
namespace {

constexpr int kG = 4;
constexpr int kXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kXor2 = 0x4E;  // quad_perm [2,3,0,1]

__device__ __forceinline__ float qxor1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kXor1, 0xF, 0xF, false));
}
__device__ __forceinline__ float qxor2(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kXor2, 0xF, 0xF, false));
}

struct BaseArgs {
  int W, H;
  const uint32_t* off;
  const float* depth;
  const void* rgba;
  float bg0, bg1, bg2;
  float* rgb;
};

// w(z, a) * a: the weight already carries one factor a, and the accumulated
// colour is the premultiplied a c
__device__ __forceinline__ float wboit_wa(float z, float a) {
  const float u = 1.0f - z;
  return a * a * fmaxf(1e-2f, 3e3f * u * u * u);
}

template <bool HALF>
__global__ __launch_bounds__(256) void wboit_kernel(BaseArgs a) {
  const int P = a.W * a.H;
  const int q = threadIdx.x & (kG - 1);
  const int p = (int)((blockIdx.x * (unsigned)blockDim.x + threadIdx.x) / kG);
  if (p >= P) return;  // whole quads leave together
  const uint32_t b = a.off[p], e = a.off[p + 1];
  float ar = 0.f, ag = 0.f, ab = 0.f, wa = 0.f, rev = 1.f;
  uint32_t k = b + q;
  for (; k + kG < e; k += 2 * kG) {
    const float z0 = a.depth[k], z1 = a.depth[k + kG];
    const float4 c0 = load_rgba<HALF>(a.rgba, k), c1 = load_rgba<HALF>(a.rgba, k + kG);
    const float a0 = __builtin_amdgcn_fmed3f(c0.w, 0.0f, 1.0f), a1 = __builtin_amdgcn_fmed3f(c1.w, 0.0f, 1.0f);
    const float w0 = wboit_wa(z0, a0), w1 = wboit_wa(z1, a1);
    ar += w0 * c0.x + w1 * c1.x;
    ag += w0 * c0.y + w1 * c1.y;
    ab += w0 * c0.z + w1 * c1.z;
    wa += w0 + w1;
    rev *= (1.0f - a0) * (1.0f - a1);
  }
  if (k < e) {
    const float z0 = a.depth[k];
    const float4 c0 = load_rgba<HALF>(a.rgba, k);
    const float a0 = __builtin_amdgcn_fmed3f(c0.w, 0.0f, 1.0f);
    const float w0 = wboit_wa(z0, a0);
    ar += w0 * c0.x;
    ag += w0 * c0.y;
    ab += w0 * c0.z;
    wa += w0;
    rev *= 1.0f - a0;
  }
  ar += qxor1(ar); ag += qxor1(ag); ab += qxor1(ab); wa += qxor1(wa); rev *= qxor1(rev);
  ar += qxor2(ar); ag += qxor2(ag); ab += qxor2(ab); wa += qxor2(wa); rev *= qxor2(rev);
  // lane q < 3 writes channel q: a quad's 12 bytes are contiguous
  if (q < 3) {
    const float acc = q == 0 ? ar : (q == 1 ? ag : ab);
    const float bgc = q == 0 ? a.bg0 : (q == 1 ? a.bg1 : a.bg2);
    const float ratio = wa > 0.0f ? acc / wa : 0.0f;
    a.rgb[3 * (size_t)p + q] = ratio * (1.0f - rev) + rev * bgc;
  }
}

// (C, T) o (C', T') = (C + T C', T T'): the first operand is in front
struct Over {
  float r, g, b, t;
};
__device__ __forceinline__ Over over(const Over& f, const Over& k) {
  return Over{fmaf(f.t, k.r, f.r), fmaf(f.t, k.g, f.g), fmaf(f.t, k.b, f.b), f.t * k.t};
}

template <bool HALF>
__global__ __launch_bounds__(256) void over_list_kernel(BaseArgs a) {
  const int P = a.W * a.H;
  const int q = threadIdx.x & (kG - 1);
  const int p = (int)((blockIdx.x * (unsigned)blockDim.x + threadIdx.x) / kG);
  if (p >= P) return;
  const uint32_t b = a.off[p], e = a.off[p + 1];
  Over run{0.f, 0.f, 0.f, 1.f};
  // the trip count depends on the pixel only, so the whole quad iterates together
  for (uint32_t k0 = b; k0 < e; k0 += kG) {
    const uint32_t k = k0 + q;
    Over m{0.f, 0.f, 0.f, 1.f};  // identity for lanes past the end
    if (k < e) {
      const float4 c = load_rgba<HALF>(a.rgba, k);
      const float al = __builtin_amdgcn_fmed3f(c.w, 0.0f, 1.0f);
      m = Over{al * c.x, al * c.y, al * c.z, 1.0f - al};
    }
    // in-quad scan in list order: pairs (0,1), (2,3), then the two pairs
    Over o{qxor1(m.r), qxor1(m.g), qxor1(m.b), qxor1(m.t)};
    m = (q & 1) ? over(o, m) : over(m, o);
    o = Over{qxor2(m.r), qxor2(m.g), qxor2(m.b), qxor2(m.t)};
    m = (q & 2) ? over(o, m) : over(m, o);
    run = over(run, m);
  }
  if (q < 3) {
    const float c = q == 0 ? run.r : (q == 1 ? run.g : run.b);
    const float bgc = q == 0 ? a.bg0 : (q == 1 ? a.bg1 : a.bg2);
    a.rgb[3 * (size_t)p + q] = fmaf(run.t, bgc, c);
  }
}

}  // namespace

int launch_baseline(const starnt_frags& f, int32_t method, const float bg[3], float* rgb, hipStream_t s) {
  BaseArgs a;
  a.W = f.width;
  a.H = f.height;
  a.off = f.offsets;
  a.depth = f.depth;
  a.rgba = f.rgba;
  a.bg0 = bg[0];
  a.bg1 = bg[1];
  a.bg2 = bg[2];
  a.rgb = rgb;
  const int P = f.width * f.height;
  const dim3 block(256), grid((unsigned)(((int64_t)P * kG + 255) / 256));
  const bool half = f.rgba_dtype == STARNT_F16;
  if (method == STARNT_BASE_WBOIT) {
    if (half) hipLaunchKernelGGL(wboit_kernel<true>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(wboit_kernel<false>, grid, block, 0, s, a);
  } else {
    if (half) hipLaunchKernelGGL(over_list_kernel<true>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(over_list_kernel<false>, grid, block, 0, s, a);
  }
  STARNT_LAUNCH_CHECK("starnt_baseline launch");
  return STARNT_OK;
}

}  // namespace starnt
