/*
 * starnt.h - C ABI of libstarnt.so, the MI355X (gfx950) per-pixel hot path of
 * STAR-NT neural order-independent transparency (Tsopouridis et al., arXiv
 * 2606.16747, "STAR-NT: Spatiotemporal Acceleration of Real-Time Neural
 * Transparency Rendering").
 *
 * Input is a frame's transparent fragments as per-pixel lists in CSR form (the
 * role the paper's rasterisation passes play). The calls are:
 *
 *   starnt_features   passes 1-3 (Sec. 3, Fig. 1): nearest layer at full
 *                     resolution, second layer on the pass-2 grid, tail
 *                     statistics and the five network features on the pass-3
 *                     grid (Sec. 3.2-3.3)
 *   starnt_infer      tail-colour network f(x) at full resolution over the
 *                     bilinearly upscaled pass-3 features (Sec. 3.2-3.3);
 *                     starnt_infer_composite fuses it with eq (3), and with a
 *                     DFAOIT network (eq (2)); starnt_infer_composite_sel runs
 *                     the network only off the flat quadtree leaves
 *   starnt_dfa_inputs the ten-feature DFAOIT input (Sec. 3.3)
 *   starnt_composite  eq (3), C = C_exact,2 + T2 f(x) + prod(1-a) C_b, with the
 *                     upscaled pass-2 layer; or the exact A-buffer composite
 *                     (eq (1) after a per-pixel sort; the paper's ground truth)
 *   starnt_quadtree   screen-tile quadtree update from the composite (Sec. 3.1)
 *                     and the pass scales of the next frame (Sec. 3.2, eq (4))
 *   starnt_reproject  interpolated frame by depth reprojection (Sec. 3.3)
 *   starnt_reproject_check, starnt_patch
 *                     its trust test and the re-rendering of untrusted pixels
 *   starnt_train_step one MSE + Adam step of the tail network (Sec. 3.3)
 *   starnt_baseline   weighted blended OIT or over in stored order (Sec. 4)
 *   starnt_interval_init / _next / _report
 *                     host policy choosing real or interpolated frames from
 *                     measured frame costs (Sec. 3.3)
 *
 * Conventions for every call:
 *  - Memory: all array arguments are DEVICE pointers owned by the caller unless
 *    marked "host". The library keeps no pointer after a call returns. No call
 *    allocates device memory; scratch comes from a caller workspace whose size
 *    starnt_workspace_size() reports.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream). Every call
 *    only enqueues work on that stream and returns without synchronising; the
 *    outputs are valid once the stream reaches that point.
 *  - Status: each call returns STARNT_OK or an error code. Arguments are
 *    validated on the host before anything is enqueued (EINVAL). Faults of the
 *    data itself (depth outside [0,1], alpha outside [0,1], a list longer than
 *    the declared maximum) are found by the kernels, which OR flags into a
 *    caller-provided device error word; read it after synchronising and pass it
 *    to starnt_check(). starnt_last_error() gives a message for the calling
 *    thread's most recent failure.
 *  - Pixels are row-major, p = y * width + x, y = 0 the top row.
 */
#ifndef STARNT_H
#define STARNT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define STARNT_OK 0
#define STARNT_EINVAL 1       /* bad argument: NULL, size, dtype, capacity     */
#define STARNT_ERANGE 2       /* data outside the documented domain            */
#define STARNT_ENOMEM 3       /* workspace smaller than starnt_workspace_size  */
#define STARNT_EHIP 4         /* a HIP launch or runtime call failed           */
#define STARNT_EUNSUPPORTED 5 /* valid but not implemented combination         */

/* device error word flags (OR-ed by kernels) */
#define STARNT_DERR_DEPTH 1u  /* a depth outside [0,1] or NaN                  */
#define STARNT_DERR_ALPHA 2u  /* an alpha outside [0,1] or NaN, among the
                                 fragments whose colour the call reads: every
                                 fragment in the exact composite; in
                                 starnt_features the two selected layers of
                                 every pixel and every fragment of a pass-3
                                 sample (the colour of other fragments is never
                                 loaded, which is what a reduced pass 3 saves) */
#define STARNT_DERR_COUNT 4u  /* a list longer than max_per_pixel              */
#define STARNT_DERR_LIST 8u   /* starnt_patch: a listed pixel outside the frame
                                 or a list longer than its capacity           */

/* ---- element types -------------------------------------------------------- */
#define STARNT_F32 0
#define STARNT_F16 1
#define STARNT_BF16 2
#define STARNT_FP8 3          /* OCP E4M3 (max 448), per-layer scales          */

/* ---- fragment lists --------------------------------------------------------
 * Pixel p owns fragments offsets[p] .. offsets[p+1]-1 (offsets[0] = 0,
 * non-decreasing, offsets[P] = num_frags). Colour is straight (not
 * premultiplied) RGBA. (depth, prim) must be unique within a pixel: the order
 * of a pixel's fragments is ascending depth with ties broken by ascending
 * primitive id, so results do not depend on the order of a list. */
typedef struct {
  int32_t width, height;
  const uint32_t* offsets;  /* [P+1]                                         */
  const float* depth;       /* [F]   NDC depth, 0 = near plane, 1 = far      */
  const void* rgba;         /* [F][4] float (STARNT_F32) or half (STARNT_F16) */
  int32_t rgba_dtype;       /* STARNT_F32 | STARNT_F16                       */
  const uint32_t* prim;     /* [F]   primitive id (read on depth ties only)  */
  uint64_t num_frags;       /* F (< 2^32)                                    */
  uint32_t max_per_pixel;   /* declared bound on list length (>= 1)          */
} starnt_frags;

/* ---- frame schedule (device resident, 64 bytes) ----------------------------
 * Grid sizes of passes 2 and 3 for the frame being rendered, and what the last
 * quadtree update measured. starnt_quadtree overwrites it with the next frame's
 * grids (eq (4)); starnt_sched_init() sets it explicitly. Grid W_s x H_s
 * samples full-resolution pixel floor((2i+1) W / (2 W_s)) along each axis. */
typedef struct {
  int32_t w2, h2, w3, h3;   /* pass-2 / pass-3 grids, 1 <= w <= width etc.  */
  uint32_t hist[4];         /* occupied quadtree leaves per level 0..3       */
  float wbar, s2, s3;       /* complexity index and the two pass scales      */
  uint32_t frames;          /* quadtree updates so far                        */
  uint32_t pad[4];
} starnt_sched;

/* ---- per-pixel intermediates written by starnt_features ------------------- */
typedef struct {
  int32_t width, height; /* frame size (must match the fragment lists)          */
  float* d1;          /* [P]    depth of layer 1; 1.0 when the list is empty    */
  float* layer1;      /* [P][4] (a1 c1r, a1 c1g, a1 c1b, a1), zero when empty   */
  uint32_t* count;    /* [P]    list length N                                   */
  float* layer2;      /* [P][4] capacity; (a2 c2, a2) at pass-2 grid samples,
                         row-major over the w2 x h2 grid                        */
  float* tail;        /* [P][8] capacity; per pass-3 grid sample:
                         x = (N, t_tail, Ct_r, Ct_g, Ct_b), then A, T2, 0, where
                         over sorted positions 3..N: A = sum a,
                         t_tail = prod (1 - a), Ct = sum a c / A (0 if A = 0),
                         and T2 = (1 - a1)(1 - a2) of the sample's two
                         selected layers (1 where it has none)                 */
  uint32_t* sel;      /* optional [P][2]: global index of layers 1 and 2
                         (0xFFFFFFFF when absent); NULL to skip                 */
  uint32_t* err;      /* device error word (flags OR-ed in; caller zeroes it)   */
  float* tail_avg;    /* optional [P][4] capacity; per pass-3 grid sample the
                         plain tail means (sum c / (N-2), sum a / (N-2)), 0
                         when N <= 2: inputs of the DFAOIT network (Sec. 3.3);
                         NULL to skip (then no extra work)                      */
} starnt_feats;

/* ---- tail-colour network ----------------------------------------------------
 * Three dense layers, ReLU after each (Sec. 3.3; the paper's widths are 32, 16;
 * any h1, h2 <= 64 with in = 16, out = 3 here). Weights are FP32 masters in
 * the layout W_l[out][in] row-major; `dtype` selects the arithmetic:
 * STARNT_F32 (VALU FP32), STARNT_BF16 (bf16 operands on the matrix cores, FP32
 * accumulate; the hidden-layer biases join that sum exactly, as three bf16
 * parts each), STARNT_FP8 (E4M3 operands with per-layer scales, FP32
 * accumulate). Input x = (N, t_tail, Ct_rgb) padded with 11 zeros. */
typedef struct {
  int32_t in, h1, h2, out;
  int32_t dtype;
  const float *W1, *b1, *W2, *b2, *W3, *b3;
  const float* fp8_scales;  /* host [6]: sa1, sw1, sa2, sw2, sa3, sw3 (FP8 only):
                               layer l computes (sum q(a/sa) q(W/sw)) sa sw + b  */
  int32_t variant;          /* STARNT_NET_STARNT (5 inputs, ReLU output, the
                               tail colour; default 0) or STARNT_NET_DFAOIT (the
                               ten-feature network STAR-NT builds on, Sec. 3.3:
                               11 inputs, sigmoid output, the whole transparent
                               colour C_t of eq (2))                            */
} starnt_mlp;
#define STARNT_NET_STARNT 0
#define STARNT_NET_DFAOIT 1

/* ---- composite modes ---------------------------------------------------- */
#define STARNT_MODE_LEARNED 0 /* f = tail_rgb from starnt_infer                 */
#define STARNT_MODE_F0 1      /* f = 0                                          */
#define STARNT_MODE_FAVG 2    /* f = Ct (1 - t_tail)                            */
#define STARNT_MODE_EXACT 3   /* exact A-buffer: per-pixel sort, eq (1)         */

/* ---- quadtree parameters (Sec. 3.1) --------------------------------------- */
typedef struct {
  int32_t base;        /* base tile size in px, multiple of 8 (paper: 16)       */
  float tau_split;     /* an unsplit node splits when D > tau_split            */
  float tau_merge;     /* a split node merges when D < tau_merge (< tau_split) */
  int32_t k_relax;     /* balance relaxation iterations (paper: 2), 0..8        */
} starnt_qt_params;

/* ---- training (Sec. 3.3: MSE, Adam) -------------------------------------- */
typedef struct {
  int32_t in, h1, h2, out;  /* in = 16, out = 3; h1, h2 in {16, 32, 64} with
                               (h1, h2) one of (16,16) (16,32) (32,16) (32,32)
                               (32,64) (64,32) (64,64); FP8: h1, h2 in {32, 64} */
  int32_t dtype;            /* STARNT_F32 (check mode) | STARNT_BF16 |
                               STARNT_FP8 (forward products on E4M3 operands,
                               backward in bf16 on the same values)           */
  float* params;            /* [n] FP32 masters: W1[h1][in], b1[h1], W2[h2][h1],
                               b2[h2], W3[out][h2], b3[out]                     */
  float* m;                 /* [n] Adam first moment                            */
  float* v;                 /* [n] Adam second moment                           */
  float* grad;              /* [n] written: gradient of this step's loss        */
  int32_t out_act;          /* output activation: 0 ReLU (STAR-NT), 1 logistic
                               sigmoid (DFAOIT); hidden layers are ReLU         */
  const float* weight;      /* [batch] optional per-sample loss weight w_k
                               (NULL: 1): loss = sum_k w_k |f(x_k) - y_k|^2 /
                               (3 batch); w = T2^2 gives the squared error of
                               eq (3)'s tail term T2 f                          */
  float fp8_act_scale[3];   /* FP8: scale s_l of layer l's input (the network
                               input, then the two hidden activations), each a
                               positive power of two: the operand is the E4M3
                               value of a / s_l (saturated at 448). Weight
                               scales are derived from the masters each step:
                               the smallest power of two s with max|W_l| / s
                               <= 448. Ignored in the other modes.            */
} starnt_train;

typedef struct {
  float lr, beta1, beta2, eps;
  int32_t step;             /* 1-based Adam step (bias correction)             */
} starnt_adam;

/* workspace kinds for starnt_workspace_size(kind, a, b, c):
 *   STARNT_WS_QUADTREE   starnt_quadtree:        a = W, b = H, c = base
 *   STARNT_WS_TRAIN      starnt_train_step:      a = batch, b = h1, c = h2
 *   STARNT_WS_REPROJECT  starnt_reproject_check: a = W, b = H (c unused) */
#define STARNT_WS_QUADTREE 1
#define STARNT_WS_TRAIN 2
#define STARNT_WS_REPROJECT 3

/* ======================================================================== */

/* Passes 1-3 over the fragment lists (Sec. 3; tail statistics and features
 * Sec. 3.3). Every pixel gets d1, layer1 and count. Pixels sampled by the
 * pass-2 grid of `sched` also get layer2, pixels sampled by the pass-3 grid get
 * a tail record. sched == NULL means both grids at full resolution. Layer
 * selection is by (depth, prim); the tail sums are exact fixed-point sums, so
 * every output is independent of the order within a list. */
int starnt_features(const starnt_frags* frags, const starnt_sched* sched, const starnt_feats* out,
                    void* stream);

/* Tail colour at full resolution (Sec. 3.3): for each pixel with count >= 3,
 * x is the bilinear upscale (half-pixel centres, clamp to edge) of the tail
 * records on the pass-3 grid of `sched` (NULL = full resolution) and
 * tail_rgb[p] = f(x); tail_rgb[p] = 0 where count < 3. tail_rgb is [P][3].
 * STARNT_NET_STARNT networks only (EINVAL for DFAOIT: it needs the layers). */
int starnt_infer(const starnt_mlp* mlp, const float* tail, const uint32_t* count, const starnt_sched* sched,
                 int32_t width, int32_t height, float* tail_rgb, void* stream);

/* starnt_infer followed by starnt_composite(STARNT_MODE_LEARNED) in one pass
 * (same results): per pixel the upscaled features feed the network and its
 * output goes straight into eq (3), so the tail colour is never stored.
 * Frame size from feats; rgb is [P][3]; bg is a host float[3].
 * With a STARNT_NET_DFAOIT network (needs feats->tail_avg) the input is the
 * upscaled DFAOIT vector of starnt_dfa_inputs and the result is eq (2):
 * C = C_t + C_b (1 - a1)(1 - a2) t_tail, with C_t the network output where
 * count >= 3 and the exact two-layer colour a1 c1 + (1 - a1) a2 c2 elsewhere. */
int starnt_infer_composite(const starnt_mlp* mlp, const starnt_feats* feats, const starnt_sched* sched,
                           const float* bg, float* rgb, void* stream);

/* Spatially selective inference (future work of the paper, Sec. 5):
 * starnt_infer_composite with a STARNT_NET_STARNT network, except that pixels
 * in a level-0 (flat) leaf of `level` take the order-free tail estimate
 * f = f_avg = Ct (1 - t_tail) instead of the network, and a 64-pixel step
 * whose pixels all have that, or no tail, skips the network. level
 * [Cw * Ch] is a quadtree leaf-level map (starnt_quadtree, base tile `base`
 * px, cells of base / 8 px, Cw = ceil(W / (base / 8))), normally the last
 * real frame's. */
int starnt_infer_composite_sel(const starnt_mlp* mlp, const starnt_feats* feats, const starnt_sched* sched,
                               const uint8_t* level, int32_t base, const float* bg, float* rgb, void* stream);

/* The DFAOIT network input of every pixel (Sec. 3.3), x [P][16] float, zero
 * where count < 3: (exact two-layer colour a1 c1 + (1 - a1) a2 c2, tail mean
 * colour, tail mean opacity, tail accumulated colour S = Ct A, N, 0 x 5), with
 * layer 2 and the pass-3 quantities upscaled from their grids as in eq (3)
 * (S per grid sample, then upscaled). Needs feats->tail_avg. Used to build
 * training pairs for STARNT_NET_DFAOIT networks. */
int starnt_dfa_inputs(const starnt_feats* feats, const starnt_sched* sched, float* x, void* stream);

/* Final colour rgb [P][3].
 * MODE_LEARNED / F0 / FAVG (eq (3), Sec. 3.3): with layer 2 and x upscaled
 *   from their grids, and the full-resolution count gating them (no layer 2
 *   where N < 2, no tail where N < 3),
 *   C = a1 c1 + (1 - a1) a2 c2 + T2 f + T2 t_tail C_b, T2 = (1 - a1)(1 - a2).
 *   Reads feats->layer1, layer2, tail, count (frame size from feats);
 *   `frags` may be NULL.
 * MODE_EXACT: sorts each list by (depth, prim) and composites front to back,
 *   C = sum_j a_j c_j prod_{k<j} (1 - a_k) + prod_j (1 - a_j) C_b (eq (1));
 *   optional fstar [P][3] receives the exact tail colour, sorted positions
 *   3..N composited alone. Reads only `frags` (+ feats->err for flags).
 *   frags->max_per_pixel (at most 2048, else EUNSUPPORTED) picks the batch
 *   size, the smallest of 192, 256 and 384 fragments that holds it; lists
 *   longer than 384 take a slower block-wide kernel, so a tight declared
 *   maximum is faster. Outputs do not depend on that choice beyond FP32
 *   rounding of the transmittance (within 1e-4 of eq (1) in FP64). A list
 *   longer than the declared maximum sets STARNT_DERR_COUNT; if it is also
 *   longer than the batch size chosen, its pixel gets the background alone.
 * bg is a host float[3]. */
int starnt_composite(const starnt_frags* frags, const starnt_feats* feats, const float* tail_rgb,
                     const starnt_sched* sched, const float* bg, int32_t mode, float* rgb, float* fstar,
                     void* stream);

/* Cheap approximate baselines of the evaluation (Sec. 4), for quality per
 * millisecond on the same fragment lists; rgb [P][3], bg a host float[3].
 * STARNT_BASE_WBOIT: weighted blended OIT (McGuire and Bavoil 2013) with the
 *   window-depth weight w(z, a) = a max(1e-2, 3e3 (1 - z)^3),
 *   C = (sum w a c / sum w a)(1 - R) + R C_b, R = prod (1 - a) (the ratio is 0
 *   when sum w a = 0). Order independent.
 * STARNT_BASE_OVER_LIST: eq (1) applied to each list in stored order with no
 *   sort (the naive blend whose error is the paper's E_random).
 * Alpha is clamped to [0, 1]; no device error word (depth or alpha outside
 *   the domain give meaningless colours, never a fault). Reads offsets, depth
 *   and rgba; prim may be NULL. */
#define STARNT_BASE_WBOIT 0
#define STARNT_BASE_OVER_LIST 1
int starnt_baseline(const starnt_frags* frags, int32_t method, const float* bg, float* rgb, void* stream);

/* Quadtree update from a real frame's composite rgb [P][3] and counts [P]
 * (Sec. 3.1): per base tile, the corner-sample distance D of every internal
 * node (mean of the six pairwise Euclidean RGB distances of its corners),
 * top-down split/merge with hysteresis against prev_mask (NULL on the first
 * frame: split iff D > tau_split, no temporal limit), leaf levels limited to
 * +-1 from prev_mask, then k_relax raise-only relaxations
 * r(c) = max(L(c), max over 4-neighbours L(n) - 1) on the global grid of
 * base/8-px cells, each followed by re-deriving masks (a node at level l is
 * split iff some cell under it has r > l).
 * Outputs: mask [Tw*Th] 21-bit split masks (bit 0 root, bits 1-4 level 1,
 * bits 5-20 level 2, Morton order), level [Cw*Ch] leaf level per cell,
 * sched->hist (occupied leaves per level), sched->wbar = sum l N_l / sum N_l,
 * sched->s2, s3 by eq (4) and the next frame's grids. The update reads and
 * writes `sched` on the device, so frames chain without host round trips.
 * Workspace: starnt_workspace_size(STARNT_WS_QUADTREE, W, H, base) bytes,
 * 256-byte aligned (EINVAL otherwise). */
int starnt_quadtree(const float* rgb, const uint32_t* count, int32_t width, int32_t height,
                    const starnt_qt_params* params, const uint32_t* prev_mask, uint32_t* mask, uint8_t* level,
                    starnt_sched* sched, void* workspace, size_t workspace_bytes, void* stream);

/* starnt_quadtree without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, outputs and errors as
 * starnt_quadtree, except that the scratch is a fixed 4 MiB array in device
 * memory that the library holds per GPU until the process ends (enough for
 * frames up to 8192 x 8192 at base 64). A frame and base whose scratch
 * (starnt_workspace_size(STARNT_WS_QUADTREE, W, H, base)) exceeds 4 MiB is
 * rejected with STARNT_ENOMEM. Allocates nothing; the first call on a device
 * looks up that device's copy of the array. Every call on a GPU shares its
 * array (no part of it needs to start at zero): calls that overlap in time
 * on one GPU, on any streams, race and give undefined results. */
int starnt_quadtree_noalloc(const float* rgb, const uint32_t* count, int32_t width, int32_t height,
                            const starnt_qt_params* params, const uint32_t* prev_mask, uint32_t* mask,
                            uint8_t* level, starnt_sched* sched, void* stream);

/* Interpolated frame (Sec. 3.3): for each pixel p, X = (x_ndc, y_ndc, d1_prev[p],
 * 1) with x_ndc = (2px+1)/W - 1, y_ndc = 1 - (2py+1)/H; h = X + (M - I) X with
 * M = VP_prev VP_cur^-1; source q = (floor((u+1) W / 2), floor((1-v) H / 2)),
 * (u, v) = (h_x, h_y) / h_w. rgb_out[p] = rgb_prev[q], src[p] = q; outside the
 * frame the source is clamped to the nearest edge pixel and src[p] = -1; when
 * h_w <= 0, src[p] = -1 and rgb_out[p] = rgb_prev[p].
 * m_minus_i is a host float[16], row-major, acting on column vectors.
 * src may be NULL. rgb_out must not overlap rgb_prev or d1_prev (EINVAL). */
int starnt_reproject(const float* rgb_prev, const float* d1_prev, int32_t width, int32_t height,
                     const float* m_minus_i, float* rgb_out, int32_t* src, void* stream);

/* Interpolated frame with a trust test (Sec. 3.3: pixels the reprojection
 * cannot fill are rendered afresh). Same gather as starnt_reproject, plus a
 * depth test at the source: with z' = h_z / h_w the reprojected depth,
 * src[p] = -2 where |d1_prev[q] - z'| > depth_tol (the source shows another
 * surface); depth_tol = 0 disables the test. The pixels with src[p] < 0 are
 * written to list (device uint32 [width*height], the caller's) in increasing
 * pixel order, and *list_count (device uint32) receives their number; the
 * compaction is deterministic (no atomics). src may be NULL; depth_tol must
 * be finite and >= 0; rgb_out must not overlap rgb_prev or d1_prev (EINVAL).
 * Workspace: starnt_workspace_size(STARNT_WS_REPROJECT, W, H, 0) bytes,
 * 256-byte aligned (EINVAL otherwise; ENOMEM when smaller). */
int starnt_reproject_check(const float* rgb_prev, const float* d1_prev, int32_t width, int32_t height,
                           const float* m_minus_i, float depth_tol, float* rgb_out, int32_t* src, uint32_t* list,
                           uint32_t* list_count, void* workspace, size_t workspace_bytes, void* stream);

/* Re-render the listed pixels of a frame from its fragment lists (Sec. 3.3,
 * the untrusted pixels of an interpolated frame): passes 1-3 at full
 * resolution and the STAR-NT network with the eq (3) composite, for pixel
 * list[i] of frags, i < min(*list_count, capacity) (list must hold that
 * many entries; list_count is a device uint32); rgb[list[i]] is overwritten and every
 * other pixel of rgb is left as it is. Each pixel's result equals that of
 * starnt_features + starnt_infer_composite at full resolution on the same
 * frame, whatever the list's order.
 * slots is scratch of the caller: a starnt_feats of width = capacity, height 1
 * (d1, layer1, count, layer2, tail and err required; sel optional), whose
 * slot i receives the features of list[i]. A count above the capacity is
 * clamped and entries outside the frame are skipped; both set
 * STARNT_DERR_LIST in slots->err. The DFAOIT network is not supported here
 * (EUNSUPPORTED). */
int starnt_patch(const starnt_frags* frags, const starnt_mlp* mlp, const uint32_t* list,
                 const uint32_t* list_count, const starnt_feats* slots, const float* bg, float* rgb, void* stream);

/* One training step on a batch (Sec. 3.3): loss = mean over batch x 3 of
 * (f(x) - y)^2 (ReLU derivative 0 at 0), gradient into t->grad, then Adam on
 * the FP32 masters with bias correction for step hp->step.
 * x [batch][16] float features, y [batch][3] float targets, loss [1] float
 * written on the device. Gradient sums over the batch use a fixed reduction
 * order, so a step is bitwise reproducible. dtype STARNT_BF16 rounds every
 * product operand (weights, inputs, activations, output gradients) to bf16
 * with FP32 accumulation; with h1 and h2 in {32, 64} the products run on the
 * matrix cores. dtype STARNT_F32 computes in FP32.
 * Workspace: starnt_workspace_size(STARNT_WS_TRAIN, batch, h1, h2). */
int starnt_train_step(const starnt_train* t, const float* x, const float* y, int32_t batch,
                      const starnt_adam* hp, float* loss, void* workspace, size_t workspace_bytes,
                      void* stream);

/* ---- host helpers (no GPU work) ------------------------------------------ */

/* Set sched to grids (ceil(s2 W), ceil(s2 H), ceil(s3 W), ceil(s3 H)), each at
 * least 1, on the device (a one-thread kernel on `stream`; hist etc. zeroed). */
int starnt_sched_init(starnt_sched* sched, int32_t width, int32_t height, double s2, double s3, void* stream);

/* wbar = sum l N_l / sum N_l over l = 0..3 (0 when all zero) (Sec. 3.2) */
double starnt_wbar(const uint32_t* hist4);
/* eq (4): s2 = clamp(2^(wbar - 2.2), 0.25, 1), s3 = clamp(2^(wbar - 3.0), 0.25, 1) */
void starnt_pass_scales(double wbar, double* s2, double* s3);
/* grid size max(1, min(n, ceil(s n))) */
int32_t starnt_grid_dim(int32_t n, double s);
/* The reprojection matrix of an interpolated frame (Sec. 3.3), in the form
 * starnt_reproject takes: out = M - I with M = vp_prev vp_cur^-1, computed in
 * FP64 (inverse by Gauss-Jordan elimination with partial pivoting) and
 * rounded to FP32. vp_prev, vp_cur: host row-major 4x4 view-projection
 * matrices of the last real frame and of the current frame; out: host
 * float[16]. Returns STARNT_EINVAL for NULL arguments or a singular vp_cur. */
int starnt_m_minus_i(const double* vp_prev, const double* vp_cur, float* out);

/* Adaptive interpolation interval (Sec. 3.3, interpolated frames): one real
 * render is followed by interval - 1 interpolated frames, interval <= 4. The
 * interval is chosen from the measured frame costs at the start of each
 * interval: the smallest k in 1..max_interval whose mean frame time
 * (real + (k - 1) interp) / k meets target_ms; k = 1 when a real frame alone
 * meets it, and also (standard rendering, no interpolation) when even
 * max_interval cannot meet it. Until an interpolated frame has been measured,
 * a real frame that misses the target is followed by a probing interval of 2.
 * Costs are running means: m <- m + smoothing (sample - m), the first sample
 * taken as is. Host only; the caller owns the struct. */
typedef struct {
  double target_ms;     /* frame-time target, 1000 / target fps; > 0        */
  double smoothing;     /* weight of a new sample in the running means, (0, 1] */
  double real_ms;       /* running mean cost of a real frame (< 0: none yet)  */
  double interp_ms;     /* running mean cost of an interpolated frame (< 0)   */
  int32_t max_interval; /* 1..4                                             */
  int32_t interval;     /* current interval (1 = every frame real)          */
  int32_t pos;          /* frames of the current interval already issued    */
  int32_t pad;
} starnt_interval;

/* Reset s; EINVAL for target_ms <= 0, smoothing outside (0, 1] or
 * max_interval outside 1..4. */
int starnt_interval_init(starnt_interval* s, double target_ms, int32_t max_interval, double smoothing);
/* Kind of the next frame: 1 = real render, 0 = interpolated (from the last
 * real frame). A new interval starts, and is re-chosen, at every real frame.
 * Returns -1 for a NULL s. */
int starnt_interval_next(starnt_interval* s);
/* Record the measured cost of a finished frame of the given kind.
 * EINVAL for a NULL s or a negative or non-finite time. */
int starnt_interval_report(starnt_interval* s, int32_t was_real, double ms);

/* bytes of workspace a call needs (a, b, c as listed at each call) */
size_t starnt_workspace_size(int32_t kind, int64_t a, int64_t b, int64_t c);

/* status for a device error word read back after the stream synchronised */
int starnt_check(uint32_t err_word);

/* Kernel timing, for callers that measure a kernel alone (a benchmark's
 * roofline, not part of the method). The next of these kernels that the
 * calling thread launches: the fragment pass (starnt_features), the network
 * (every call that runs it) or the exact path's main kernel (starnt_composite
 * with STARNT_MODE_EXACT), goes out through hipExtLaunchKernel, which records
 * start_event when the kernel starts and stop_event when it ends, so their
 * elapsed time is the kernel's own duration, without the dispatch gaps of
 * events recorded around the call. Both are hipEvent_t created (and recorded
 * once) by the caller with timing enabled; either may be NULL. The request
 * holds for that one launch and is then cleared; both NULL clears it. Meant
 * for eager launches: leave no request pending while capturing a HIP graph.
 * Never fails. */
int starnt_time_next_launch(void* start_event, void* stop_event);

/* message of the calling thread's last failure ("" if none) */
const char* starnt_last_error(void);

/* library version, e.g. "starnt 0.1 gfx950" */
const char* starnt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STARNT_H */
