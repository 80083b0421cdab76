// C ABI of libstarnt: argument validation on the host, then the launchers.
// Every function enqueues on the caller's stream and returns without waiting.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace starnt {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_status(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return STARNT_EHIP;
}

static thread_local LaunchTimer g_timer;

LaunchTimer take_launch_timer() {
  const LaunchTimer t = g_timer;
  g_timer = LaunchTimer();
  return t;
}

}  // namespace starnt

using namespace starnt;

namespace {

constexpr int64_t kMaxSide = 16384;

int check_frame(int32_t W, int32_t H, const char* who) {
  if (W <= 0 || H <= 0 || W > kMaxSide || H > kMaxSide)
    return fail(STARNT_EINVAL, std::string(who) + ": width/height must be in [1, 16384]");
  return STARNT_OK;
}

int check_frags(const starnt_frags* f, const char* who) {
  if (!f) return fail(STARNT_EINVAL, std::string(who) + ": frags is NULL");
  int rc = check_frame(f->width, f->height, who);
  if (rc) return rc;
  if (!f->offsets) return fail(STARNT_EINVAL, std::string(who) + ": offsets is NULL");
  if (f->num_frags > 0 && (!f->depth || !f->rgba || !f->prim))
    return fail(STARNT_EINVAL, std::string(who) + ": NULL fragment array");
  if (f->rgba_dtype != STARNT_F32 && f->rgba_dtype != STARNT_F16)
    return fail(STARNT_EINVAL, std::string(who) + ": rgba_dtype must be STARNT_F32 or STARNT_F16");
  if (f->num_frags >= (1ull << 32))
    return fail(STARNT_EINVAL, std::string(who) + ": num_frags must be below 2^32");
  if (f->max_per_pixel == 0) return fail(STARNT_EINVAL, std::string(who) + ": max_per_pixel must be >= 1");
  return STARNT_OK;
}

int check_mlp(const starnt_mlp* mlp, const char* who) {
  const std::string w(who);
  if (!mlp) return fail(STARNT_EINVAL, w + ": NULL network");
  if (mlp->in != 16 || mlp->out != 3) return fail(STARNT_EINVAL, w + ": the network must have in = 16 and out = 3");
  if (mlp->h1 < 1 || mlp->h1 > 64 || mlp->h2 < 1 || mlp->h2 > 64)
    return fail(STARNT_EINVAL, w + ": hidden widths must be in [1, 64]");
  if (!mlp->W1 || !mlp->b1 || !mlp->W2 || !mlp->b2 || !mlp->W3 || !mlp->b3)
    return fail(STARNT_EINVAL, w + ": NULL weight array");
  if (mlp->dtype != STARNT_F32 && mlp->dtype != STARNT_BF16 && mlp->dtype != STARNT_FP8)
    return fail(STARNT_EINVAL, w + ": dtype must be STARNT_F32, STARNT_BF16 or STARNT_FP8");
  if (mlp->dtype == STARNT_FP8 && !mlp->fp8_scales) return fail(STARNT_EINVAL, w + ": FP8 needs fp8_scales");
  if (mlp->fp8_scales)
    for (int i = 0; i < 6; ++i)
      if (!(mlp->fp8_scales[i] > 0.0f) || !std::isfinite(mlp->fp8_scales[i]))
        return fail(STARNT_EINVAL, w + ": fp8 scales must be finite and positive");
  if (mlp->variant != STARNT_NET_STARNT && mlp->variant != STARNT_NET_DFAOIT)
    return fail(STARNT_EINVAL, w + ": variant must be STARNT_NET_STARNT or STARNT_NET_DFAOIT");
  return STARNT_OK;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

int starnt_features(const starnt_frags* frags, const starnt_sched* sched, const starnt_feats* out,
                    void* stream) {
  int rc = check_frags(frags, "starnt_features");
  if (rc) return rc;
  if (!out || !out->d1 || !out->layer1 || !out->count || !out->layer2 || !out->tail || !out->err)
    return fail(STARNT_EINVAL, "starnt_features: NULL output array (d1, layer1, count, layer2, tail, err)");
  if (out->width != frags->width || out->height != frags->height)
    return fail(STARNT_EINVAL, "starnt_features: feats and frags differ in width/height");
  return launch_features(*frags, sched, *out, as_stream(stream));
}

int starnt_infer(const starnt_mlp* mlp, const float* tail, const uint32_t* count, const starnt_sched* sched,
                 int32_t width, int32_t height, float* tail_rgb, void* stream) {
  int rc = check_frame(width, height, "starnt_infer");
  if (rc) return rc;
  if (!tail || !count || !tail_rgb) return fail(STARNT_EINVAL, "starnt_infer: NULL argument");
  rc = check_mlp(mlp, "starnt_infer");
  if (rc) return rc;
  if (mlp->variant != STARNT_NET_STARNT)
    return fail(STARNT_EINVAL, "starnt_infer: a DFAOIT network needs the layers (starnt_infer_composite)");
  return launch_infer(*mlp, tail, count, sched, width, height, tail_rgb, as_stream(stream));
}

int starnt_infer_composite(const starnt_mlp* mlp, const starnt_feats* feats, const starnt_sched* sched,
                           const float* bg, float* rgb, void* stream) {
  if (!feats) return fail(STARNT_EINVAL, "starnt_infer_composite: NULL feats");
  int rc = check_frame(feats->width, feats->height, "starnt_infer_composite");
  if (rc) return rc;
  if (!bg || !rgb || !feats->layer1 || !feats->count || !feats->layer2 || !feats->tail)
    return fail(STARNT_EINVAL, "starnt_infer_composite: NULL argument");
  rc = check_mlp(mlp, "starnt_infer_composite");
  if (rc) return rc;
  if (mlp->variant == STARNT_NET_DFAOIT && !feats->tail_avg)
    return fail(STARNT_EINVAL, "starnt_infer_composite: a DFAOIT network needs feats->tail_avg");
  return launch_infer_composite(*mlp, *feats, sched, bg, rgb, as_stream(stream));
}

int starnt_infer_composite_sel(const starnt_mlp* mlp, const starnt_feats* feats, const starnt_sched* sched,
                               const uint8_t* level, int32_t base, const float* bg, float* rgb, void* stream) {
  if (!feats) return fail(STARNT_EINVAL, "starnt_infer_composite_sel: NULL feats");
  int rc = check_frame(feats->width, feats->height, "starnt_infer_composite_sel");
  if (rc) return rc;
  if (!bg || !rgb || !level || !feats->layer1 || !feats->count || !feats->layer2 || !feats->tail)
    return fail(STARNT_EINVAL, "starnt_infer_composite_sel: NULL argument");
  if (base < 8 || base % 8 || base > 4096)
    return fail(STARNT_EINVAL, "starnt_infer_composite_sel: base must be a multiple of 8 in [8, 4096]");
  rc = check_mlp(mlp, "starnt_infer_composite_sel");
  if (rc) return rc;
  if (mlp->variant != STARNT_NET_STARNT)
    return fail(STARNT_EINVAL, "starnt_infer_composite_sel: STAR-NT networks only");
  return launch_infer_composite_sel(*mlp, *feats, sched, level, base, bg, rgb, as_stream(stream));
}

int starnt_dfa_inputs(const starnt_feats* feats, const starnt_sched* sched, float* x, void* stream) {
  if (!feats) return fail(STARNT_EINVAL, "starnt_dfa_inputs: NULL feats");
  int rc = check_frame(feats->width, feats->height, "starnt_dfa_inputs");
  if (rc) return rc;
  if (!x || !feats->layer1 || !feats->count || !feats->layer2 || !feats->tail || !feats->tail_avg)
    return fail(STARNT_EINVAL, "starnt_dfa_inputs: NULL argument (x, layer1, count, layer2, tail, tail_avg)");
  return launch_dfa_inputs(*feats, sched, x, as_stream(stream));
}

int starnt_composite(const starnt_frags* frags, const starnt_feats* feats, const float* tail_rgb,
                     const starnt_sched* sched, const float* bg, int32_t mode, float* rgb, float* fstar,
                     void* stream) {
  if (!bg || !rgb) return fail(STARNT_EINVAL, "starnt_composite: NULL bg or rgb");
  if (mode == STARNT_MODE_EXACT) {
    int rc = check_frags(frags, "starnt_composite");
    if (rc) return rc;
    uint32_t* err = feats ? feats->err : nullptr;
    return launch_exact(*frags, bg, rgb, fstar, err, as_stream(stream));
  }
  if (mode != STARNT_MODE_LEARNED && mode != STARNT_MODE_F0 && mode != STARNT_MODE_FAVG)
    return fail(STARNT_EINVAL, "starnt_composite: unknown mode");
  if (!feats || !feats->layer1 || !feats->count || !feats->layer2 || !feats->tail)
    return fail(STARNT_EINVAL, "starnt_composite: NULL feature array");
  if (mode == STARNT_MODE_LEARNED && !tail_rgb)
    return fail(STARNT_EINVAL, "starnt_composite: learned mode needs tail_rgb");
  const int W = feats->width, H = feats->height;
  int rc = check_frame(W, H, "starnt_composite");
  if (rc) return rc;
  return launch_composite(*feats, tail_rgb, sched, W, H, bg, mode, rgb, as_stream(stream));
}

int starnt_baseline(const starnt_frags* frags, int32_t method, const float* bg, float* rgb, void* stream) {
  if (!frags) return fail(STARNT_EINVAL, "starnt_baseline: frags is NULL");
  int rc = check_frame(frags->width, frags->height, "starnt_baseline");
  if (rc) return rc;
  if (!frags->offsets) return fail(STARNT_EINVAL, "starnt_baseline: offsets is NULL");
  if (frags->num_frags > 0 && (!frags->depth || !frags->rgba))
    return fail(STARNT_EINVAL, "starnt_baseline: NULL fragment array");
  if (frags->rgba_dtype != STARNT_F32 && frags->rgba_dtype != STARNT_F16)
    return fail(STARNT_EINVAL, "starnt_baseline: rgba_dtype must be STARNT_F32 or STARNT_F16");
  if (frags->num_frags >= (1ull << 32)) return fail(STARNT_EINVAL, "starnt_baseline: num_frags must be below 2^32");
  if (!bg || !rgb) return fail(STARNT_EINVAL, "starnt_baseline: NULL bg or rgb");
  if (method != STARNT_BASE_WBOIT && method != STARNT_BASE_OVER_LIST)
    return fail(STARNT_EINVAL, "starnt_baseline: unknown method");
  return launch_baseline(*frags, method, bg, rgb, as_stream(stream));
}

static int check_quadtree(const float* rgb, const uint32_t* count, int32_t width, int32_t height,
                          const starnt_qt_params* params, const uint32_t* prev_mask, const uint32_t* mask,
                          const uint8_t* level, const starnt_sched* sched, const char* who) {
  const std::string w(who);
  int rc = check_frame(width, height, who);
  if (rc) return rc;
  if (!rgb || !count || !params || !mask || !level || !sched) return fail(STARNT_EINVAL, w + ": NULL argument");
  if (params->base < 8 || params->base % 8 || params->base > 4096)
    return fail(STARNT_EINVAL, w + ": base must be a multiple of 8 in [8, 4096]");
  if (params->k_relax < 0 || params->k_relax > 8) return fail(STARNT_EINVAL, w + ": k_relax must be in [0, 8]");
  if (!(params->tau_merge <= params->tau_split))
    return fail(STARNT_EINVAL, w + ": tau_merge must not exceed tau_split");
  if (prev_mask && prev_mask == mask) return fail(STARNT_EINVAL, w + ": prev_mask aliases mask");
  return STARNT_OK;
}

int starnt_quadtree(const float* rgb, const uint32_t* count, int32_t width, int32_t height,
                    const starnt_qt_params* params, const uint32_t* prev_mask, uint32_t* mask, uint8_t* level,
                    starnt_sched* sched, void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_quadtree(rgb, count, width, height, params, prev_mask, mask, level, sched, "starnt_quadtree");
  if (rc) return rc;
  const size_t need = quadtree_ws_bytes(width, height, params->base);
  if (!workspace || workspace_bytes < need) return fail(STARNT_ENOMEM, "starnt_quadtree: workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(STARNT_EINVAL, "starnt_quadtree: workspace must be 256-byte aligned");
  return launch_quadtree(rgb, count, width, height, *params, prev_mask, mask, level, sched, workspace,
                         as_stream(stream));
}

int starnt_quadtree_noalloc(const float* rgb, const uint32_t* count, int32_t width, int32_t height,
                            const starnt_qt_params* params, const uint32_t* prev_mask, uint32_t* mask,
                            uint8_t* level, starnt_sched* sched, void* stream) {
  int rc = check_quadtree(rgb, count, width, height, params, prev_mask, mask, level, sched,
                          "starnt_quadtree_noalloc");
  if (rc) return rc;
  return launch_quadtree_noalloc(rgb, count, width, height, *params, prev_mask, mask, level, sched,
                                 as_stream(stream));
}

// [a, a + na) and [b, b + nb) share a byte (addresses compared as integers)
static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}
// the gather's output [P][3] against its inputs rgb [P][3] and d1 [P]
static bool gather_overlaps(const float* rgb, const float* d1, const float* out, int32_t w, int32_t h) {
  const size_t P = (size_t)w * (size_t)h;
  return ranges_overlap(out, 12 * P, rgb, 12 * P) || ranges_overlap(out, 12 * P, d1, 4 * P);
}

int starnt_reproject(const float* rgb_prev, const float* d1_prev, int32_t width, int32_t height,
                     const float* m_minus_i, float* rgb_out, int32_t* src, void* stream) {
  int rc = check_frame(width, height, "starnt_reproject");
  if (rc) return rc;
  if (!rgb_prev || !d1_prev || !m_minus_i || !rgb_out) return fail(STARNT_EINVAL, "starnt_reproject: NULL argument");
  if (gather_overlaps(rgb_prev, d1_prev, rgb_out, width, height))
    return fail(STARNT_EINVAL, "starnt_reproject: rgb_out overlaps rgb_prev or d1_prev");
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(m_minus_i[i])) return fail(STARNT_EINVAL, "starnt_reproject: non-finite matrix");
  return launch_reproject(rgb_prev, d1_prev, width, height, m_minus_i, rgb_out, src, as_stream(stream));
}

int starnt_reproject_check(const float* rgb_prev, const float* d1_prev, int32_t width, int32_t height,
                           const float* m_minus_i, float depth_tol, float* rgb_out, int32_t* src, uint32_t* list,
                           uint32_t* list_count, void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_frame(width, height, "starnt_reproject_check");
  if (rc) return rc;
  if (!rgb_prev || !d1_prev || !m_minus_i || !rgb_out || !list || !list_count)
    return fail(STARNT_EINVAL, "starnt_reproject_check: NULL argument");
  if (gather_overlaps(rgb_prev, d1_prev, rgb_out, width, height))
    return fail(STARNT_EINVAL, "starnt_reproject_check: rgb_out overlaps rgb_prev or d1_prev");
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(m_minus_i[i])) return fail(STARNT_EINVAL, "starnt_reproject_check: non-finite matrix");
  if (!std::isfinite(depth_tol) || depth_tol < 0.0f)
    return fail(STARNT_EINVAL, "starnt_reproject_check: depth_tol must be finite and >= 0");
  if (!workspace) return fail(STARNT_EINVAL, "starnt_reproject_check: NULL workspace");
  if (workspace_bytes < reproject_ws_bytes(width, height))
    return fail(STARNT_ENOMEM, "starnt_reproject_check: workspace smaller than starnt_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail(STARNT_EINVAL, "starnt_reproject_check: workspace must be 256-byte aligned");
  return launch_reproject(rgb_prev, d1_prev, width, height, m_minus_i, rgb_out, src, as_stream(stream), depth_tol,
                          list, list_count, workspace);
}

int starnt_patch(const starnt_frags* frags, const starnt_mlp* mlp, const uint32_t* list,
                 const uint32_t* list_count, const starnt_feats* slots, const float* bg, float* rgb, void* stream) {
  int rc = check_frags(frags, "starnt_patch");
  if (rc) return rc;
  rc = check_mlp(mlp, "starnt_patch");
  if (rc) return rc;
  if (mlp->variant != STARNT_NET_STARNT)
    return fail(STARNT_EUNSUPPORTED, "starnt_patch: only the STAR-NT network re-renders pixel lists");
  if (!list || !list_count || !bg || !rgb) return fail(STARNT_EINVAL, "starnt_patch: NULL argument");
  if (!slots || !slots->d1 || !slots->layer1 || !slots->count || !slots->layer2 || !slots->tail || !slots->err)
    return fail(STARNT_EINVAL, "starnt_patch: NULL slot array (d1, layer1, count, layer2, tail, err)");
  if (slots->height != 1 || slots->width < 1)
    return fail(STARNT_EINVAL, "starnt_patch: slots must be a 1-row block (width = capacity, height = 1)");
  const hipStream_t s = as_stream(stream);
  rc = launch_features_list(*frags, list, list_count, *slots, s);
  if (rc) return rc;
  return launch_infer_patch(*mlp, *slots, list, list_count, (uint32_t)frags->width * (uint32_t)frags->height, bg,
                            rgb, s);
}

int starnt_train_step(const starnt_train* t, const float* x, const float* y, int32_t batch,
                      const starnt_adam* hp, float* loss, void* workspace, size_t workspace_bytes,
                      void* stream) {
  if (!t || !x || !y || !hp || !loss) return fail(STARNT_EINVAL, "starnt_train_step: NULL argument");
  if (!t->params || !t->m || !t->v || !t->grad) return fail(STARNT_EINVAL, "starnt_train_step: NULL state array");
  if (t->in != 16 || t->out != 3) return fail(STARNT_EINVAL, "starnt_train_step: in must be 16 and out 3");
  if (t->dtype != STARNT_F32 && t->dtype != STARNT_BF16 && t->dtype != STARNT_FP8)
    return fail(STARNT_EINVAL, "starnt_train_step: dtype must be STARNT_F32, STARNT_BF16 or STARNT_FP8");
  if (t->dtype == STARNT_FP8) {
    for (int l = 0; l < 3; ++l) {
      int e = 0;
      const float v = t->fp8_act_scale[l];
      if (!(v > 0.0f) || !std::isfinite(v) || std::frexp(v, &e) != 0.5f)
        return fail(STARNT_EINVAL, "starnt_train_step: FP8 activation scales must be positive powers of two");
    }
  }
  if (batch < 1 || batch > (1 << 24)) return fail(STARNT_EINVAL, "starnt_train_step: batch must be in [1, 2^24]");
  if (hp->step < 1) return fail(STARNT_EINVAL, "starnt_train_step: Adam step is 1-based");
  if (t->out_act != 0 && t->out_act != 1) return fail(STARNT_EINVAL, "starnt_train_step: out_act must be 0 or 1");
  if (!(hp->beta1 >= 0.0f && hp->beta1 < 1.0f && hp->beta2 >= 0.0f && hp->beta2 < 1.0f))
    return fail(STARNT_EINVAL, "starnt_train_step: betas must be in [0, 1)");
  const size_t need = train_ws_bytes(batch, t->h1, t->h2);
  if (!workspace || workspace_bytes < need) return fail(STARNT_ENOMEM, "starnt_train_step: workspace too small");
  return launch_train(*t, x, y, batch, *hp, loss, workspace, workspace_bytes, as_stream(stream));
}

int starnt_sched_init(starnt_sched* sched, int32_t width, int32_t height, double s2, double s3, void* stream) {
  int rc = check_frame(width, height, "starnt_sched_init");
  if (rc) return rc;
  if (!sched) return fail(STARNT_EINVAL, "starnt_sched_init: NULL sched");
  if (!(s2 > 0.0 && s2 <= 1.0 && s3 > 0.0 && s3 <= 1.0))
    return fail(STARNT_EINVAL, "starnt_sched_init: scales must be in (0, 1]");
  return launch_sched_init(sched, starnt_grid_dim(width, s2), starnt_grid_dim(height, s2),
                           starnt_grid_dim(width, s3), starnt_grid_dim(height, s3), as_stream(stream));
}

double starnt_wbar(const uint32_t* h) {
  if (!h) return 0.0;
  const double den = (double)h[0] + h[1] + h[2] + h[3];
  return den > 0 ? ((double)h[1] + 2.0 * h[2] + 3.0 * h[3]) / den : 0.0;
}

void starnt_pass_scales(double wbar, double* s2, double* s3) {
  const double a = std::exp2(wbar - 2.2), b = std::exp2(wbar - 3.0);
  if (s2) *s2 = std::fmin(1.0, std::fmax(0.25, a));
  if (s3) *s3 = std::fmin(1.0, std::fmax(0.25, b));
}

int starnt_m_minus_i(const double* vp_prev, const double* vp_cur, float* out) {
  if (!vp_prev || !vp_cur || !out) return fail(STARNT_EINVAL, "starnt_m_minus_i: NULL argument");
  // [vp_cur | I] reduced to [I | vp_cur^-1], largest pivot of each column
  double a[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 8; ++c) a[r][c] = c < 4 ? vp_cur[4 * r + c] : (c - 4 == r ? 1.0 : 0.0);
  double scale = 0.0;
  for (int i = 0; i < 16; ++i) scale = std::fmax(scale, std::fabs(vp_cur[i]));
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
    if (!(std::fabs(a[piv][c]) > 1e-300 + 1e-14 * scale))
      return fail(STARNT_EINVAL, "starnt_m_minus_i: vp_cur is singular");
    if (piv != c)
      for (int k = 0; k < 8; ++k) std::swap(a[c][k], a[piv][k]);
    const double inv = 1.0 / a[c][c];
    for (int k = 0; k < 8; ++k) a[c][k] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      for (int k = 0; k < 8; ++k) a[r][k] -= f * a[c][k];
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double m = 0.0;
      for (int k = 0; k < 4; ++k) m += vp_prev[4 * r + k] * a[k][4 + c];
      out[4 * r + c] = (float)(m - (r == c ? 1.0 : 0.0));
    }
  return STARNT_OK;
}

int32_t starnt_grid_dim(int32_t n, double s) {
  double v = std::ceil(s * (double)n);
  v = std::fmax(1.0, std::fmin((double)n, v));
  return (int32_t)v;
}

size_t starnt_workspace_size(int32_t kind, int64_t a, int64_t b, int64_t c) {
  if (kind == STARNT_WS_QUADTREE) return quadtree_ws_bytes(a, b, c);
  if (kind == STARNT_WS_TRAIN) return train_ws_bytes(a, b, c);
  if (kind == STARNT_WS_REPROJECT) return reproject_ws_bytes(a, b);
  return 0;
}

int starnt_check(uint32_t err_word) {
  if (!err_word) return STARNT_OK;
  std::string m = "device error word:";
  if (err_word & STARNT_DERR_DEPTH) m += " depth outside [0,1];";
  if (err_word & STARNT_DERR_ALPHA) m += " alpha outside [0,1];";
  if (err_word & STARNT_DERR_COUNT) m += " list longer than max_per_pixel;";
  if (err_word & STARNT_DERR_LIST) m += " pixel list entry outside the frame or longer than its capacity;";
  return fail(STARNT_ERANGE, m);
}

int starnt_time_next_launch(void* start_event, void* stop_event) {
  g_timer.start = static_cast<hipEvent_t>(start_event);
  g_timer.stop = static_cast<hipEvent_t>(stop_event);
  return STARNT_OK;
}

const char* starnt_last_error(void) { return g_last_error.c_str(); }

const char* starnt_version(void) { return "starnt 0.1 gfx950"; }

}  // extern "C"
