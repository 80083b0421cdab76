/*
 * Plain FP64 CPU oracle for the STAR-NT per-pixel path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code with the GPU path.
 *
 * Every routine is the plain definition written out with loops in double
 * precision: sort each pixel's fragments, walk them front to back, evaluate the
 * network one scalar at a time. No blocking, fusion or reordering beyond what
 * the definitions state. Citations are to the STAR-NT paper (arXiv 2606.16747):
 *   eq (1)  Porter-Duff over, front to back (Sec. 3.2)
 *   eq (3)  decoupled composite C = C_exact,2 + T2 f(x) + prod(1-a) C_b (Sec. 3.3)
 *   eq (4)  pass scale s_p = clamp(2^(wbar - delta_p), 0.25, 1) (Sec. 3.2)
 *   Sec. 3.1 quadtree of screen tiles, corner-sample distance D, hysteresis,
 *            top-down refinement, +-1 level per frame, k = 2 relaxations
 *   Sec. 3.3 five-float input (N, t_tail, normalised tail colour), MLP with
 *            ReLU output trained with MSE and Adam; interpolated frames by
 *            depth reprojection with the previous view-projection.
 *
 * Where the paper leaves a point open, the reading taken is stated at the
 * routine that uses it. Parity pins for each function live in tests/.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Per-pixel order: ascending (depth, primitive id).                          */

typedef struct {
  double z;
  uint32_t prim;
  double a, r, g, b;
} frag_t;

static int key_less(const frag_t* x, const frag_t* y) {
  if (x->z != y->z) return x->z < y->z;
  return x->prim < y->prim;
}

/* insertion sort: plain and obviously correct; lists are at most a few hundred */
static void sort_frags(frag_t* f, int n) {
  for (int i = 1; i < n; ++i) {
    frag_t t = f[i];
    int j = i - 1;
    while (j >= 0 && key_less(&t, &f[j])) {
      f[j + 1] = f[j];
      --j;
    }
    f[j + 1] = t;
  }
}

static int load_pixel(const uint32_t* off, const float* depth, const float* rgba, const uint32_t* prim,
                      int64_t p, frag_t* buf, int32_t* pos) {
  uint32_t b = off[p], e = off[p + 1];
  int n = (int)(e - b);
  for (int k = 0; k < n; ++k) {
    uint32_t i = b + (uint32_t)k;
    buf[k].z = depth[i];
    buf[k].prim = prim[i];
    buf[k].a = rgba[4 * (size_t)i + 3];
    buf[k].r = rgba[4 * (size_t)i + 0];
    buf[k].g = rgba[4 * (size_t)i + 1];
    buf[k].b = rgba[4 * (size_t)i + 2];
  }
  (void)pos;
  return n;
}

/* global fragment index of the fragment at sorted position j (for selection checks) */
static uint32_t find_index(const uint32_t* off, const float* depth, const uint32_t* prim, int64_t p,
                           const frag_t* f) {
  for (uint32_t i = off[p]; i < off[p + 1]; ++i)
    if ((double)depth[i] == f->z && prim[i] == f->prim) return i;
  return 0xFFFFFFFFu;
}

/*
 * Per-pixel quantities of one frame, all at full resolution.
 *
 * rgb   [P][3]  exact A-buffer composite over background bg (eq (1) with
 *               premultiplied colour alpha*c, then T_N * C_b)
 * fstar [P][3]  exact tail colour: the fragments at sorted positions 3..N
 *               composited alone, no background
 * lay   [P][10] N, d1, a1, c1(3), a2, c2(3); a missing layer has a = c = 0,
 *               d1 = 1 when N = 0
 * tail  [P][6]  A = sum a, S = sum a*c (3), t_tail = prod (1-a), Ctilde
 *               is not stored (S/A); tail = sorted positions 3..N
 * sel   [P][2]  global fragment index of layer 1 and layer 2 (0xFFFFFFFF if none)
 * tavg  [P][4]  plain means over the tail (sorted positions 3..N): colour
 *               sum c / (N-2) and opacity sum a / (N-2); 0 when N <= 2
 *               (inputs of the DFAOIT network, Sec. 3.3)
 * Any output pointer may be NULL.
 */
int orc_frame(int32_t W, int32_t H, const uint32_t* off, const float* depth, const float* rgba,
              const uint32_t* prim, const double* bg, double* rgb, double* fstar, double* lay, double* tail,
              uint32_t* sel, double* tavg, int32_t nthreads) {
  int64_t P = (int64_t)W * H;
  uint32_t maxn = 0;
  for (int64_t p = 0; p < P; ++p) {
    uint32_t n = off[p + 1] - off[p];
    if (n > maxn) maxn = n;
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    frag_t* f = (frag_t*)malloc(sizeof(frag_t) * (maxn + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
    for (int64_t p = 0; p < P; ++p) {
      int n = load_pixel(off, depth, rgba, prim, p, f, NULL);
      sort_frags(f, n);
      /* eq (1): C = sum_j T_{j-1} a_j c_j, T_j = T_{j-1} (1 - a_j) */
      double T = 1.0, C[3] = {0, 0, 0};
      for (int j = 0; j < n; ++j) {
        C[0] += T * f[j].a * f[j].r;
        C[1] += T * f[j].a * f[j].g;
        C[2] += T * f[j].a * f[j].b;
        T *= (1.0 - f[j].a);
      }
      if (rgb) {
        rgb[3 * p + 0] = C[0] + T * bg[0];
        rgb[3 * p + 1] = C[1] + T * bg[1];
        rgb[3 * p + 2] = C[2] + T * bg[2];
      }
      /* exact tail colour: positions 3..N composited alone */
      if (fstar) {
        double Tt = 1.0, Ft[3] = {0, 0, 0};
        for (int j = 2; j < n; ++j) {
          Ft[0] += Tt * f[j].a * f[j].r;
          Ft[1] += Tt * f[j].a * f[j].g;
          Ft[2] += Tt * f[j].a * f[j].b;
          Tt *= (1.0 - f[j].a);
        }
        fstar[3 * p + 0] = Ft[0];
        fstar[3 * p + 1] = Ft[1];
        fstar[3 * p + 2] = Ft[2];
      }
      if (lay) {
        double* L = lay + 10 * p;
        L[0] = n;
        L[1] = n > 0 ? f[0].z : 1.0;
        L[2] = n > 0 ? f[0].a : 0.0;
        L[3] = n > 0 ? f[0].r : 0.0;
        L[4] = n > 0 ? f[0].g : 0.0;
        L[5] = n > 0 ? f[0].b : 0.0;
        L[6] = n > 1 ? f[1].a : 0.0;
        L[7] = n > 1 ? f[1].r : 0.0;
        L[8] = n > 1 ? f[1].g : 0.0;
        L[9] = n > 1 ? f[1].b : 0.0;
      }
      if (tail) {
        double A = 0, S[3] = {0, 0, 0}, t = 1.0;
        for (int j = 2; j < n; ++j) {
          A += f[j].a;
          S[0] += f[j].a * f[j].r;
          S[1] += f[j].a * f[j].g;
          S[2] += f[j].a * f[j].b;
          t *= (1.0 - f[j].a);
        }
        double* Q = tail + 6 * p;
        Q[0] = A;
        Q[1] = S[0];
        Q[2] = S[1];
        Q[3] = S[2];
        Q[4] = t;
        Q[5] = 0.0;
      }
      if (tavg) {
        double sc[3] = {0, 0, 0}, sa = 0;
        for (int j = 2; j < n; ++j) {
          sc[0] += f[j].r;
          sc[1] += f[j].g;
          sc[2] += f[j].b;
          sa += f[j].a;
        }
        double* Q = tavg + 4 * p;
        for (int c = 0; c < 3; ++c) Q[c] = n > 2 ? sc[c] / (n - 2) : 0.0;
        Q[3] = n > 2 ? sa / (n - 2) : 0.0;
      }
      if (sel) {
        sel[2 * p + 0] = n > 0 ? find_index(off, depth, prim, p, &f[0]) : 0xFFFFFFFFu;
        sel[2 * p + 1] = n > 1 ? find_index(off, depth, prim, p, &f[1]) : 0xFFFFFFFFu;
      }
    }
    free(f);
  }
  return 0;
}

/*
 * Five network features of a pixel from its tail statistics (Sec. 3.3):
 *   x = [N, t_tail, Ctilde_r, Ctilde_g, Ctilde_b],
 *   t_tail = prod over the tail of (1 - a)  (1 for an empty tail),
 *   Ctilde = sum a c / sum a                 (0 when sum a = 0).
 * Reading: the paper's alpha_acc is taken as the tail transmittance for the
 * t_tail feature and as the tail opacity sum for the normalisation of Ctilde.
 */
static void features_from(double N, const double* tail6, double* x5) {
  double A = tail6[0];
  x5[0] = N;
  x5[1] = tail6[4];
  for (int c = 0; c < 3; ++c) x5[2 + c] = A > 0 ? tail6[1 + c] / A : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Network: three dense layers, ReLU after each (Sec. 3.3). W_l is [out][in].  */

typedef struct {
  int32_t in, h1, h2, out;
  const float *W1, *b1, *W2, *b2, *W3, *b3;
} orc_mlp;

static void dense_relu(int nin, int nout, const float* W, const float* b, const double* x, double* y) {
  for (int o = 0; o < nout; ++o) {
    double s = b[o];
    for (int i = 0; i < nin; ++i) s += (double)W[(size_t)o * nin + i] * x[i];
    y[o] = s > 0.0 ? s : 0.0;
  }
}

/* Output activation: act 0 ReLU (STAR-NT, Sec. 3.3), act 1 logistic sigmoid
 * (the DFAOIT network the paper starts from, Sec. 3.3). Hidden layers are
 * ReLU in both. */
static double out_act(double z, int32_t act) { return act ? 1.0 / (1.0 + exp(-z)) : (z > 0.0 ? z : 0.0); }

/* y[n][out] = f(x[n][in]) in FP64 */
int orc_mlp_forward_act(const orc_mlp* m, const double* x, int64_t n, int32_t act, double* y) {
  if (m->h1 > 1024 || m->h2 > 1024 || m->out > 64 || m->in > 64) return -1;
  for (int64_t k = 0; k < n; ++k) {
    double h1[1024], h2[1024];
    dense_relu(m->in, m->h1, m->W1, m->b1, x + (size_t)k * m->in, h1);
    dense_relu(m->h1, m->h2, m->W2, m->b2, h1, h2);
    for (int o = 0; o < m->out; ++o) {
      double s = m->b3[o];
      for (int i = 0; i < m->h2; ++i) s += (double)m->W3[(size_t)o * m->h2 + i] * h2[i];
      y[(size_t)k * m->out + o] = out_act(s, act);
    }
  }
  return 0;
}

int orc_mlp_forward(const orc_mlp* m, const double* x, int64_t n, double* y) {
  return orc_mlp_forward_act(m, x, n, 0, y);
}

/* ---- reduced-precision operands (used only to state per-layer error) ---- */

/* bfloat16 round-to-nearest-even of an FP32 value: keep the high 16 bits of
 * the IEEE-754 single after adding half an ulp (ties to even). */
static double round_bf16(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return v;  /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  u &= 0xFFFF0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

/* OCP FP8 E4M3 ("e4m3fn": bias 7, no infinities, max finite 448) with
 * round-to-nearest-even and saturation to +-448. Value set: subnormals
 * m * 2^-9 (m = 0..7), normals (1 + m/8) * 2^(e-7), e = 1..15, except
 * e = 15, m = 7 (NaN). */
static double round_e4m3(double v) {
  if (v != v) return v;
  double s = v < 0 ? -1.0 : 1.0, a = fabs(v);
  if (a >= 448.0) return s * 448.0;
  /* spacing of representable values around a */
  int e;
  if (a < ldexp(1.0, -6)) {
    e = -6; /* subnormal range: spacing 2^-9 */
  } else {
    e = (int)floor(log2(a));
    if (ldexp(1.0, e) > a) e -= 1;
    if (ldexp(1.0, e + 1) <= a) e += 1;
  }
  double q = ldexp(1.0, e - 3); /* 3 mantissa bits */
  double k = a / q;
  double r = floor(k);
  double d = k - r;
  if (d > 0.5 || (d == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
  double out = r * q;
  if (out > 448.0) out = 448.0;
  return s * out;
}

double orc_round_bf16(double v) { return round_bf16(v); }
double orc_round_e4m3(double v) { return round_e4m3(v); }

/*
 * Forward pass with operands rounded to a narrow format at the points a
 * matrix engine consumes them: each layer's input activations and weights are
 * rounded (bf16: qmode 1; e4m3 with scales: qmode 2), products summed in FP64,
 * bias added in FP64, ReLU, and the next layer's input rounded again.
 * For e4m3, layer l uses activation scale sa[l] and weight scale sw[l]:
 *   y = (sum_i q(x_i / sa) q(W_oi / sw)) * sa * sw + b.
 * Biases are not rounded (a matrix engine adds them in its FP32 sum).
 * Pins (tests/test_oracle_pins_quant_mixed.py): hand-computed bf16 and e4m3
 * examples that separate a rounded bias, an unrounded layer input and scales
 * applied before the bias; equality with the FP64 forward on operands that
 * are exact in the narrow format.
 */
/* Narrow operand of layer l: bf16 (qmode 1) or e4m3 of v / scale (qmode 2). */
static double narrow(double v, int32_t qmode, double scale) {
  return qmode == 1 ? round_bf16(v) : round_e4m3(v / scale);
}

/* Forward with narrow operands. Optional amb[k]: bit 0 when an input of
 * sample k lies so close to a rounding boundary of its narrow type that
 * moving it by d = tol_in |v| changes its rounding by more than 4 d (a step of
 * the type, not a rounding of the move itself); bit 1 the same for a hidden
 * activation moved by tol_h times the sum of the absolute terms (and the
 * bias) that produce it. A computation in another precision that stays
 * within those distances rounds every operand of an unflagged sample to the
 * same value as this one, or to one within 4 d of it. Optional ymag [n][out]:
 * each output's sum of absolute terms and bias (the size its own
 * accumulation error scales with). */
int orc_mlp_forward_q_amb(const orc_mlp* m, const double* x, int64_t n, int32_t qmode, const double* sa,
                          const double* sw, int32_t act, double tol_in, double tol_h, double* y, uint8_t* amb,
                          double* ymag) {
  if (m->h1 > 1024 || m->h2 > 1024 || m->out > 64 || m->in > 64) return -1;
  const int dims[4] = {m->in, m->h1, m->h2, m->out};
  const float* Ws[3] = {m->W1, m->W2, m->W3};
  const float* bs[3] = {m->b1, m->b2, m->b3};
  for (int64_t k = 0; k < n; ++k) {
    /* a: this layer's inputs; mag: the size each input is known to (its own
       size for the network input, the sum of absolute terms for an activation) */
    double a[1024], o[1024], mag[1024], omag[1024];
    uint8_t flag = 0;
    for (int i = 0; i < m->in; ++i) {
      a[i] = x[(size_t)k * m->in + i];
      mag[i] = fabs(a[i]);
    }
    for (int l = 0; l < 3; ++l) {
      int nin = dims[l], nout = dims[l + 1];
      if (amb && qmode != 0) {
        const double tol = l == 0 ? tol_in : tol_h;
        const double scale = qmode == 2 ? sa[l] : 1.0;
        for (int i = 0; i < nin; ++i) {
          /* two roundings farther apart than the move itself: a step of the
             narrow type (operands of the size of the move, such as an
             activation at the ReLU's kink, round within it) */
          const double d = tol * mag[i];
          const double lo = narrow(a[i] - d, qmode, scale) * scale, hi = narrow(a[i] + d, qmode, scale) * scale;
          if (hi - lo > 4.0 * d) flag |= l == 0 ? 1 : 2;
        }
      }
      for (int j = 0; j < nout; ++j) {
        double s = 0.0, sabs = 0.0;
        for (int i = 0; i < nin; ++i) {
          double w = Ws[l][(size_t)j * nin + i];
          double av = a[i];
          double t;
          if (qmode == 1) {
            t = round_bf16(av) * round_bf16(w);
          } else if (qmode == 2) {
            t = round_e4m3(av / sa[l]) * round_e4m3(w / sw[l]);
          } else {
            t = av * w;
          }
          s += t;
          sabs += fabs(t);
        }
        if (qmode == 2) {
          s *= sa[l] * sw[l];
          sabs *= sa[l] * sw[l];
        }
        s += bs[l][j];
        o[j] = l == 2 ? out_act(s, act) : (s > 0.0 ? s : 0.0);
        omag[j] = sabs + fabs((double)bs[l][j]);
      }
      for (int j = 0; j < nout; ++j) {
        a[j] = o[j];
        mag[j] = omag[j];
      }
    }
    for (int j = 0; j < m->out; ++j) y[(size_t)k * m->out + j] = a[j];
    if (amb) amb[k] = flag;
    /* the output layer's sum of absolute terms (and bias), per output */
    if (ymag)
      for (int j = 0; j < m->out; ++j) ymag[(size_t)k * m->out + j] = mag[j];
  }
  return 0;
}

int orc_mlp_forward_q_act(const orc_mlp* m, const double* x, int64_t n, int32_t qmode, const double* sa,
                          const double* sw, int32_t act, double* y) {
  return orc_mlp_forward_q_amb(m, x, n, qmode, sa, sw, act, 0.0, 0.0, y, NULL, NULL);
}

int orc_mlp_forward_q(const orc_mlp* m, const double* x, int64_t n, int32_t qmode, const double* sa,
                      const double* sw, double* y) {
  return orc_mlp_forward_q_act(m, x, n, qmode, sa, sw, 0, y);
}

/* ------------------------------------------------------------------------ */
/* Mixed resolution (Sec. 3.2): passes 2 and 3 on a W_s x H_s grid.           */

/* grid size for scale s: max(1, ceil(s * W)) */
int32_t orc_grid_dim(int32_t W, double s) {
  double v = ceil(s * (double)W);
  if (v < 1.0) v = 1.0;
  if (v > (double)W) v = (double)W;
  return (int32_t)v;
}

/* full-resolution pixel sampled by grid index i: floor((2i+1) W / (2 W_s)) */
int32_t orc_sample_pos(int32_t W, int32_t Ws, int32_t i) {
  int64_t num = (int64_t)(2 * (int64_t)i + 1) * W;
  return (int32_t)(num / (2 * (int64_t)Ws));
}

/* bilinear taps for full-resolution coordinate x: grid coordinate
 * u = ((2x+1) Ws - W) / (2W) (half-pixel centres), taps clamped to the edge */
static void taps(int32_t W, int32_t Ws, int32_t x, int32_t* i0, int32_t* i1, double* fr) {
  int64_t num = (int64_t)(2 * (int64_t)x + 1) * Ws - W;
  int64_t den = 2 * (int64_t)W;
  int64_t q = num >= 0 ? num / den : -((-num + den - 1) / den);
  *fr = (double)(num - q * den) / (double)den;
  int64_t a = q, b = q + 1;
  if (a < 0) a = 0;
  if (a > Ws - 1) a = Ws - 1;
  if (b < 0) b = 0;
  if (b > Ws - 1) b = Ws - 1;
  *i0 = (int32_t)a;
  *i1 = (int32_t)b;
}

/* bilinear upscale of a [Hs][Ws][C] grid to [H][W][C] */
int orc_upsample(int32_t W, int32_t H, int32_t Ws, int32_t Hs, int32_t C, const double* g, double* out) {
  for (int32_t y = 0; y < H; ++y) {
    int32_t j0, j1;
    double fy;
    taps(H, Hs, y, &j0, &j1, &fy);
    for (int32_t x = 0; x < W; ++x) {
      int32_t i0, i1;
      double fx;
      taps(W, Ws, x, &i0, &i1, &fx);
      for (int32_t c = 0; c < C; ++c) {
        double v00 = g[((size_t)j0 * Ws + i0) * C + c], v01 = g[((size_t)j0 * Ws + i1) * C + c];
        double v10 = g[((size_t)j1 * Ws + i0) * C + c], v11 = g[((size_t)j1 * Ws + i1) * C + c];
        double top = (1.0 - fx) * v00 + fx * v01;
        double bot = (1.0 - fx) * v10 + fx * v11;
        out[((size_t)y * W + x) * C + c] = (1.0 - fy) * top + fy * bot;
      }
    }
  }
  return 0;
}

/*
 * The learned path for one real frame (Sec. 3.2-3.3), from per-pixel exact
 * quantities `lay` and `tail` produced by orc_frame:
 *   pass 1 at full resolution: layer 1 and the count N;
 *   pass 2 sampled on the W2 x H2 grid: (a2, a2*c2), upscaled bilinearly;
 *   pass 3 sampled on the W3 x H3 grid: x = [N, t_tail, Ctilde], upscaled;
 *   reading: the exact full-resolution count N gates the upscaled terms
 *   (N < 2: no second layer; N < 3: no tail, t_tail = 1, f = 0);
 *   f = MLP(x) (mode 0), f = 0 (mode 1) or f = Ctilde (1 - t_tail) (mode 2);
 *   eq (3): C = a1 c1 + (1 - a1) a2 c2 + T2 f + T2 t_tail C_b,
 *           T2 = (1 - a1)(1 - a2).
 * Outputs: rgb [P][3]; optional xf [P][16] network input (5 features + zeros),
 * optional f [P][3] tail colour used.
 * Pins at s < 1 (tests/test_oracle_pins_quant_mixed.py): identical lists give
 * the full-resolution result on any grids; hand-computed bilinear weights on a
 * 6 x 1 frame with pass-2 and pass-3 grids of different widths.
 */
int orc_learned(int32_t W, int32_t H, const double* lay, const double* tail, int32_t W2, int32_t H2, int32_t W3,
                int32_t H3, const orc_mlp* m, int32_t mode, const double* bg, double* rgb, double* xf,
                double* fout) {
  int64_t P = (int64_t)W * H;
  double* g2 = (double*)calloc((size_t)W2 * H2 * 4, sizeof(double));
  double* g3 = (double*)calloc((size_t)W3 * H3 * 5, sizeof(double));
  double* u2 = (double*)calloc((size_t)P * 4, sizeof(double));
  double* u3 = (double*)calloc((size_t)P * 5, sizeof(double));
  if (!g2 || !g3 || !u2 || !u3) {
    free(g2); free(g3); free(u2); free(u3);
    return -1;
  }
  for (int32_t j = 0; j < H2; ++j)
    for (int32_t i = 0; i < W2; ++i) {
      int64_t p = (int64_t)orc_sample_pos(H, H2, j) * W + orc_sample_pos(W, W2, i);
      const double* L = lay + 10 * p;
      double* g = g2 + ((size_t)j * W2 + i) * 4;
      g[0] = L[6];
      g[1] = L[6] * L[7];
      g[2] = L[6] * L[8];
      g[3] = L[6] * L[9];
    }
  for (int32_t j = 0; j < H3; ++j)
    for (int32_t i = 0; i < W3; ++i) {
      int64_t p = (int64_t)orc_sample_pos(H, H3, j) * W + orc_sample_pos(W, W3, i);
      features_from(lay[10 * p], tail + 6 * p, g3 + ((size_t)j * W3 + i) * 5);
    }
  orc_upsample(W, H, W2, H2, 4, g2, u2);
  orc_upsample(W, H, W3, H3, 5, g3, u3);
  int in = m ? m->in : 16;
  /* pixels are independent: the loop runs in parallel, each pixel's
     arithmetic unchanged */
#ifdef _OPENMP
#pragma omp parallel
#endif
  {
  double* xin = (double*)calloc((size_t)(in > 5 ? in : 5), sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(static, 4096)
#endif
  for (int64_t p = 0; p < P; ++p) {
    const double* L = lay + 10 * p;
    double N = L[0];
    double a1 = L[2], c1[3] = {L[3], L[4], L[5]};
    double a2 = u2[4 * p + 0], pc2[3] = {u2[4 * p + 1], u2[4 * p + 2], u2[4 * p + 3]};
    if (N < 2) {
      a2 = 0;
      pc2[0] = pc2[1] = pc2[2] = 0;
    }
    double x5[5];
    for (int c = 0; c < 5; ++c) x5[c] = u3[5 * p + c];
    double f[3] = {0, 0, 0};
    double tt = x5[1];
    if (N < 3) {
      tt = 1.0;
    } else if (mode == 0) {
      for (int c = 0; c < in; ++c) xin[c] = c < 5 ? x5[c] : 0.0;
      orc_mlp_forward(m, xin, 1, f);
    } else if (mode == 2) {
      for (int c = 0; c < 3; ++c) f[c] = x5[2 + c] * (1.0 - x5[1]);
    }
    if (xf) {
      for (int c = 0; c < 16; ++c) xf[16 * p + c] = c < 5 ? x5[c] : 0.0;
    }
    if (fout) {
      for (int c = 0; c < 3; ++c) fout[3 * p + c] = f[c];
    }
    double T2 = (1.0 - a1) * (1.0 - a2);
    for (int c = 0; c < 3; ++c)
      rgb[3 * p + c] = a1 * c1[c] + (1.0 - a1) * pc2[c] + T2 * f[c] + T2 * tt * bg[c];
  }
  free(xin);
  }
  free(g2); free(g3); free(u2); free(u3);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Quadtree (Sec. 3.1) and pass scales (Sec. 3.2, eq (4)).                     */

/* complexity index wbar = sum l N_l / sum N_l (0 when no tile is occupied) */
double orc_wbar(const uint32_t* hist4) {
  double num = 0, den = 0;
  for (int l = 0; l < 4; ++l) {
    num += (double)l * hist4[l];
    den += hist4[l];
  }
  return den > 0 ? num / den : 0.0;
}

/* eq (4): s_p = clamp(2^(wbar - delta_p), 0.25, 1), delta_2 = 2.2, delta_3 = 3.0 */
void orc_pass_scales(double wbar, double* s2, double* s3) {
  double a = pow(2.0, wbar - 2.2), b = pow(2.0, wbar - 3.0);
  *s2 = a < 0.25 ? 0.25 : (a > 1.0 ? 1.0 : a);
  *s3 = b < 0.25 ? 0.25 : (b > 1.0 ? 1.0 : b);
}

typedef struct {
  int32_t base;       /* base tile size in pixels (16 in the paper, 64 at 1080p here) */
  double tau_split;   /* an unsplit node splits when D > tau_split */
  double tau_merge;   /* a split node merges when D < tau_merge */
  int32_t k_relax;    /* relaxation iterations (2 in the paper) */
} orc_qt_params;

/* node index inside a tile's 21-bit mask: level 0 -> 0, level 1 -> 1..4,
 * level 2 -> 5..20, Morton order (x bit below y bit at each level) */
static int node_bit(int lvl, int nx, int ny) {
  if (lvl == 0) return 0;
  if (lvl == 1) return 1 + (nx + 2 * ny);
  int q1 = (nx >> 1) + 2 * (ny >> 1);
  int q2 = (nx & 1) + 2 * (ny & 1);
  return 5 + 4 * q1 + q2;
}

/* mean of the 6 pairwise Euclidean distances between a node's corner colours */
static double corner_distance(const float* rgb, int32_t W, int32_t H, int64_t x0, int64_t y0, int64_t s) {
  if (x0 >= W || y0 >= H) return 0.0;
  int64_t x1 = x0 + s - 1, y1 = y0 + s - 1;
  if (x1 > W - 1) x1 = W - 1;
  if (y1 > H - 1) y1 = H - 1;
  int64_t px[4] = {x0, x1, x0, x1}, py[4] = {y0, y0, y1, y1};
  double c[4][3];
  for (int k = 0; k < 4; ++k)
    for (int ch = 0; ch < 3; ++ch) c[k][ch] = rgb[3 * (py[k] * W + px[k]) + ch];
  double sum = 0;
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) {
      double d2 = 0;
      for (int ch = 0; ch < 3; ++ch) d2 += (c[a][ch] - c[b][ch]) * (c[a][ch] - c[b][ch]);
      sum += sqrt(d2);
    }
  return sum / 6.0;
}

/* leaf level of cell (cx, cy) under a tile mask */
static int leaf_level(uint32_t mask, int cx, int cy) {
  /* cx, cy are cell coordinates within the tile, 0..7 */
  if (!(mask & 1u)) return 0;
  if (!(mask & (1u << node_bit(1, cx >> 2, cy >> 2)))) return 1;
  if (!(mask & (1u << node_bit(2, cx >> 1, cy >> 1)))) return 2;
  return 3;
}

/*
 * One quadtree update from the final composite of a real frame.
 *
 * rgb [P][3], N [P] (fragment counts), prev_mask [T] (NULL on the first frame),
 * outputs mask [T] (21-bit split masks), level [Cw*Ch] (leaf level per
 * 8x8-cell of the base/8 grid), hist[4] (occupied leaves per level),
 * optional D [T][21], optional force [T][21] (-1 none, else the decision to
 * adopt for that node when it is evaluated; used only where the FP64 distance
 * lies within a rounding band of a threshold).
 *
 * Steps (Sec. 3.1): top-down split/merge with hysteresis from prev_mask;
 * per-cell level clamped to prev +- 1; then k raise-only Jacobi relaxations
 * r(c) = max(L(c), max over 4-neighbours L(n) - 1) on the global cell grid,
 * each followed by re-deriving the masks (a node at level l is split iff some
 * cell under it has r > l) and re-reading the leaf levels.
 */
int orc_quadtree(int32_t W, int32_t H, const float* rgb, const uint32_t* N, const orc_qt_params* qp,
                 const uint32_t* prev_mask, uint32_t* mask, uint8_t* level, uint32_t* hist, double* Dout,
                 const int8_t* force) {
  const int32_t B = qp->base;
  if (B < 8 || (B & 7)) return -1;
  const int32_t cs = B >> 3; /* cell (level-3 node) size */
  const int32_t Tw = (W + B - 1) / B, Th = (H + B - 1) / B;
  const int32_t Cw = (W + cs - 1) / cs, Ch = (H + cs - 1) / cs;
  int* L = (int*)malloc(sizeof(int) * (size_t)Cw * Ch);
  int* R = (int*)malloc(sizeof(int) * (size_t)Cw * Ch);
  if (!L || !R) {
    free(L); free(R);
    return -1;
  }
  /* top-down decisions per tile (tiles are independent: each writes only its
   * own D rows and cells; threads of the caller's OpenMP setting) */
#pragma omp parallel for collapse(2) schedule(static)
  for (int32_t ty = 0; ty < Th; ++ty)
    for (int32_t tx = 0; tx < Tw; ++tx) {
      int64_t t = (int64_t)ty * Tw + tx;
      uint32_t pm = prev_mask ? prev_mask[t] : 0u;
      uint32_t m = 0;
      for (int lvl = 0; lvl <= 2; ++lvl) {
        int n = 1 << lvl;
        int64_t s = B >> lvl;
        for (int ny = 0; ny < n; ++ny)
          for (int nx = 0; nx < n; ++nx) {
            int bit = node_bit(lvl, nx, ny);
            int64_t x0 = (int64_t)tx * B + nx * s, y0 = (int64_t)ty * B + ny * s;
            double D = corner_distance(rgb, W, H, x0, y0, s);
            if (Dout) Dout[21 * t + bit] = D;
            int considered = (lvl == 0) || (m & (1u << node_bit(lvl - 1, nx >> 1, ny >> 1)));
            if (!considered) continue;
            int split;
            if (prev_mask && (pm & (1u << bit)))
              split = !(D < qp->tau_merge);
            else
              split = D > qp->tau_split;
            if (force && force[21 * t + bit] >= 0) split = force[21 * t + bit];
            if (split) m |= 1u << bit;
          }
      }
      for (int cy = 0; cy < 8; ++cy)
        for (int cx = 0; cx < 8; ++cx) {
          int64_t gx = (int64_t)tx * 8 + cx, gy = (int64_t)ty * 8 + cy;
          if (gx >= Cw || gy >= Ch) continue;
          int lv = leaf_level(m, cx, cy);
          if (prev_mask) {
            int pl = leaf_level(pm, cx, cy);
            if (lv > pl + 1) lv = pl + 1;
            if (lv < pl - 1) lv = pl - 1;
          }
          L[gy * Cw + gx] = lv;
        }
    }
  /* masks from a level map, then leaf levels from the masks */
  for (int it = 0; it <= qp->k_relax; ++it) {
    if (it > 0) {
#pragma omp parallel for schedule(static)
      for (int32_t gy = 0; gy < Ch; ++gy)
        for (int32_t gx = 0; gx < Cw; ++gx) {
          int r = L[gy * Cw + gx];
          if (gx > 0 && L[gy * Cw + gx - 1] - 1 > r) r = L[gy * Cw + gx - 1] - 1;
          if (gx < Cw - 1 && L[gy * Cw + gx + 1] - 1 > r) r = L[gy * Cw + gx + 1] - 1;
          if (gy > 0 && L[(gy - 1) * Cw + gx] - 1 > r) r = L[(gy - 1) * Cw + gx] - 1;
          if (gy < Ch - 1 && L[(gy + 1) * Cw + gx] - 1 > r) r = L[(gy + 1) * Cw + gx] - 1;
          R[gy * Cw + gx] = r;
        }
    } else {
      memcpy(R, L, sizeof(int) * (size_t)Cw * Ch);
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int32_t ty = 0; ty < Th; ++ty)
      for (int32_t tx = 0; tx < Tw; ++tx) {
        uint32_t m = 0;
        for (int lvl = 0; lvl <= 2; ++lvl) {
          int n = 1 << lvl, span = 8 >> lvl; /* cells per node side */
          for (int ny = 0; ny < n; ++ny)
            for (int nx = 0; nx < n; ++nx) {
              int any = 0;
              for (int cy = ny * span; cy < (ny + 1) * span; ++cy)
                for (int cx = nx * span; cx < (nx + 1) * span; ++cx) {
                  int64_t gx = (int64_t)tx * 8 + cx, gy = (int64_t)ty * 8 + cy;
                  if (gx >= Cw || gy >= Ch) continue;
                  if (R[gy * Cw + gx] > lvl) any = 1;
                }
              if (any) m |= 1u << node_bit(lvl, nx, ny);
            }
        }
        /* keep only nodes whose parent chain is split (tree form) */
        uint32_t mt = 0;
        if (m & 1u) {
          mt |= 1u;
          for (int q = 0; q < 4; ++q) {
            int b1 = 1 + q;
            if (!(m & (1u << b1))) continue;
            mt |= 1u << b1;
            for (int r2 = 0; r2 < 4; ++r2) {
              int b2 = 5 + 4 * q + r2;
              if (m & (1u << b2)) mt |= 1u << b2;
            }
          }
        }
        mask[(int64_t)ty * Tw + tx] = mt;
        for (int cy = 0; cy < 8; ++cy)
          for (int cx = 0; cx < 8; ++cx) {
            int64_t gx = (int64_t)tx * 8 + cx, gy = (int64_t)ty * 8 + cy;
            if (gx >= Cw || gy >= Ch) continue;
            L[gy * Cw + gx] = leaf_level(mt, cx, cy);
          }
      }
  }
  for (int64_t c = 0; c < (int64_t)Cw * Ch; ++c) level[c] = (uint8_t)L[c];
  /* occupied leaves per level: a leaf is occupied when some pixel inside it
   * (and inside the frame) has at least one fragment */
  uint32_t h0 = 0, h1 = 0, h2 = 0, h3 = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : h0, h1, h2, h3)
  for (int32_t ty = 0; ty < Th; ++ty)
    for (int32_t tx = 0; tx < Tw; ++tx) {
      uint32_t mt = mask[(int64_t)ty * Tw + tx];
      /* enumerate leaves */
      for (int lvl = 0; lvl <= 3; ++lvl) {
        int n = 1 << lvl;
        int64_t s = B >> lvl;
        for (int ny = 0; ny < n; ++ny)
          for (int nx = 0; nx < n; ++nx) {
            /* node is a leaf iff its parent chain is split and it is not split */
            int is_leaf;
            if (lvl == 0)
              is_leaf = !(mt & 1u);
            else {
              int parent_split = (mt & (1u << node_bit(lvl - 1, nx >> 1, ny >> 1))) != 0;
              int self_split = lvl < 3 ? (mt & (1u << node_bit(lvl, nx, ny))) != 0 : 0;
              is_leaf = parent_split && !self_split;
            }
            if (!is_leaf) continue;
            int64_t x0 = (int64_t)tx * B + nx * s, y0 = (int64_t)ty * B + ny * s;
            int occ = 0;
            for (int64_t y = y0; y < y0 + s && y < H && !occ; ++y)
              for (int64_t x = x0; x < x0 + s && x < W; ++x)
                if (N[y * W + x] >= 1) {
                  occ = 1;
                  break;
                }
            if (occ) {
              if (lvl == 0) ++h0;
              else if (lvl == 1) ++h1;
              else if (lvl == 2) ++h2;
              else ++h3;
            }
          }
      }
    }
  hist[0] = h0;
  hist[1] = h1;
  hist[2] = h2;
  hist[3] = h3;
  free(L);
  free(R);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Reprojection gather (Sec. 3.3, interpolated frames).                        */

/*
 * For each pixel p of an interpolated frame t: its NDC position
 * X = ((2px+1)/W - 1, 1 - (2py+1)/H, d1_r(p), 1) with the first-fragment depth
 * of the last real frame r at the same pixel, mapped by M = VP_r VP_t^-1
 * (given as M - I, row-major, column vectors), divided by w, and rounded to the
 * nearest source pixel (floor((u+1) W / 2), floor((1-v) H / 2)).
 * Inside the frame: out[p] = rgb_r[q], src[p] = q. Outside the frame the
 * source is clamped to the nearest edge pixel (edge extension) and src[p] = -1.
 * When w <= 0 (behind the camera): src[p] = -1 and out[p] = rgb_r[p].
 * margin (optional) receives the distance, in pixels, of the source coordinate
 * to the nearest rounding boundary (either axis).
 */
int orc_reproject(int32_t W, int32_t H, const float* rgb_r, const float* d1_r, const double* mmi, float* out,
                  int32_t* src, double* margin) {
  /* rows are independent (out never aliases rgb_r): they run in parallel */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int32_t py = 0; py < H; ++py)
    for (int32_t px = 0; px < W; ++px) {
      int64_t p = (int64_t)py * W + px;
      double X[4] = {(2.0 * px + 1.0) / W - 1.0, 1.0 - (2.0 * py + 1.0) / H, (double)d1_r[p], 1.0};
      double h[4];
      for (int r = 0; r < 4; ++r) {
        h[r] = X[r];
        for (int c = 0; c < 4; ++c) h[r] += mmi[4 * r + c] * X[c];
      }
      int32_t q = -1;
      int64_t s = p;
      double mg = 1e30;
      if (h[3] > 0.0) {
        double u = h[0] / h[3], v = h[1] / h[3];
        double sx = (u + 1.0) * 0.5 * W, sy = (1.0 - v) * 0.5 * H;
        double qx = floor(sx), qy = floor(sy);
        double mx = fmin(sx - qx, qx + 1.0 - sx), my = fmin(sy - qy, qy + 1.0 - sy);
        mg = fmin(mx, my);
        if (qx >= 0 && qx < W && qy >= 0 && qy < H) q = (int32_t)((int64_t)qy * W + (int64_t)qx);
        double cx = qx < 0 ? 0 : (qx > W - 1 ? W - 1 : qx);
        double cy = qy < 0 ? 0 : (qy > H - 1 ? H - 1 : qy);
        s = (int64_t)cy * W + (int64_t)cx;
      }
      if (src) src[p] = q;
      if (margin) margin[p] = mg;
      for (int c = 0; c < 3; ++c) out[3 * p + c] = rgb_r[3 * s + c];
    }
  return 0;
}

/*
 * Trust test of the gather (selective re-rendering of interpolated frames):
 * with the same mapping as orc_reproject, code[p] = q for a source inside the
 * frame whose first-fragment depth matches the reprojected depth
 * z' = h_z / h_w within tol; -2 when it does not (a disocclusion or a depth
 * edge); -1 outside the frame or behind the camera. tol <= 0 disables the
 * depth test. zdiff (optional) receives |d1_r(q) - z'| (0 where q < 0).
 */
int orc_reproject_check(int32_t W, int32_t H, const float* d1_r, const double* mmi, double tol, int32_t* code,
                        double* zdiff) {
  for (int32_t py = 0; py < H; ++py)
    for (int32_t px = 0; px < W; ++px) {
      int64_t p = (int64_t)py * W + px;
      double X[4] = {(2.0 * px + 1.0) / W - 1.0, 1.0 - (2.0 * py + 1.0) / H, (double)d1_r[p], 1.0};
      double h[4];
      for (int r = 0; r < 4; ++r) {
        h[r] = X[r];
        for (int c = 0; c < 4; ++c) h[r] += mmi[4 * r + c] * X[c];
      }
      int32_t q = -1;
      double dz = 0.0;
      if (h[3] > 0.0) {
        double u = h[0] / h[3], v = h[1] / h[3];
        double qx = floor((u + 1.0) * 0.5 * W), qy = floor((1.0 - v) * 0.5 * H);
        if (qx >= 0 && qx < W && qy >= 0 && qy < H) {
          q = (int32_t)((int64_t)qy * W + (int64_t)qx);
          dz = fabs((double)d1_r[q] - h[2] / h[3]);
          if (tol > 0.0 && dz > tol) q = -2;
        }
      }
      code[p] = q;
      if (zdiff) zdiff[p] = dz;
    }
  return 0;
}

/* 4x4 inverse by Gauss-Jordan with partial pivoting (for the full-matrix form) */
int orc_inverse4(const double* a, double* inv) {
  double m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? a[4 * i + j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(m[r][c]) > fabs(m[piv][c])) piv = r;
    if (m[piv][c] == 0.0) return -1;
    for (int j = 0; j < 8; ++j) {
      double t = m[c][j];
      m[c][j] = m[piv][j];
      m[piv][j] = t;
    }
    double d = m[c][c];
    for (int j = 0; j < 8; ++j) m[c][j] /= d;
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        double f = m[r][c];
        for (int j = 0; j < 8; ++j) m[r][j] -= f * m[c][j];
      }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) inv[4 * i + j] = m[i][j + 4];
  return 0;
}

/* source coordinates by explicit unprojection through VP_t^-1 and projection
 * through VP_r (brute-force form, for checking the M - I form) */
int orc_reproject_full(int32_t W, int32_t H, const float* d1_r, const double* vp_r, const double* vp_t,
                       double* su, double* sv) {
  double inv[16];
  if (orc_inverse4(vp_t, inv)) return -1;
  for (int32_t py = 0; py < H; ++py)
    for (int32_t px = 0; px < W; ++px) {
      int64_t p = (int64_t)py * W + px;
      double X[4] = {(2.0 * px + 1.0) / W - 1.0, 1.0 - (2.0 * py + 1.0) / H, (double)d1_r[p], 1.0};
      double wpos[4], h[4];
      for (int r = 0; r < 4; ++r) {
        wpos[r] = 0;
        for (int c = 0; c < 4; ++c) wpos[r] += inv[4 * r + c] * X[c];
      }
      for (int r = 0; r < 4; ++r) {
        h[r] = 0;
        for (int c = 0; c < 4; ++c) h[r] += vp_r[4 * r + c] * wpos[c];
      }
      su[p] = (h[0] / h[3] + 1.0) * 0.5 * W;
      sv[p] = (1.0 - h[1] / h[3]) * 0.5 * H;
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Training (Sec. 3.3: MSE loss, Adam).                                        */

/*
 * Parameter vector layout: W1[h1][in], b1[h1], W2[h2][h1], b2[h2], W3[out][h2], b3[out].
 * Loss = mean over B*out of wt_k (f(x_k) - y_k)^2, with per-sample weights wt
 * (NULL: all 1, the plain MSE of Sec. 3.3). With wt_k = T2_k^2 this is the
 * mean squared error of the composite, since eq (3) scales f by T2.
 * grad receives dLoss/dparams. ReLU derivative at 0 is taken as 0.
 */
double orc_mlp_loss_grad_wt(const int32_t* dims, const double* w, const double* x, const double* y,
                            const double* wt, int64_t B, int32_t act, double* grad) {
  const int in = dims[0], h1 = dims[1], h2 = dims[2], out = dims[3];
  const double* W1 = w;
  const double* b1 = W1 + (size_t)h1 * in;
  const double* W2 = b1 + h1;
  const double* b2 = W2 + (size_t)h2 * h1;
  const double* W3 = b2 + h2;
  const double* b3 = W3 + (size_t)out * h2;
  size_t np = (size_t)h1 * in + h1 + (size_t)h2 * h1 + h2 + (size_t)out * h2 + out;
  if (grad) memset(grad, 0, np * sizeof(double));
  double* gW1 = grad;
  double* gb1 = grad ? gW1 + (size_t)h1 * in : NULL;
  double* gW2 = grad ? gb1 + h1 : NULL;
  double* gb2 = grad ? gW2 + (size_t)h2 * h1 : NULL;
  double* gW3 = grad ? gb2 + h2 : NULL;
  double* gb3 = grad ? gW3 + (size_t)out * h2 : NULL;
  double* z1 = (double*)malloc(sizeof(double) * (h1 + h2 + out) * 2);
  double* z2 = z1 + h1;
  double* z3 = z2 + h2;
  double* d1 = z3 + out;
  double* d2 = d1 + h1;
  double* d3 = d2 + h2;
  double loss = 0;
  const double scale = 1.0 / ((double)B * out);
  for (int64_t k = 0; k < B; ++k) {
    const double* xk = x + (size_t)k * in;
    const double* yk = y + (size_t)k * out;
    for (int o = 0; o < h1; ++o) {
      double s = b1[o];
      for (int i = 0; i < in; ++i) s += W1[(size_t)o * in + i] * xk[i];
      z1[o] = s;
    }
    for (int o = 0; o < h2; ++o) {
      double s = b2[o];
      for (int i = 0; i < h1; ++i) s += W2[(size_t)o * h1 + i] * (z1[i] > 0 ? z1[i] : 0.0);
      z2[o] = s;
    }
    for (int o = 0; o < out; ++o) {
      double s = b3[o];
      for (int i = 0; i < h2; ++i) s += W3[(size_t)o * h2 + i] * (z2[i] > 0 ? z2[i] : 0.0);
      z3[o] = s;
    }
    const double wk = wt ? wt[k] : 1.0;
    for (int o = 0; o < out; ++o) {
      double f = out_act(z3[o], act);
      double e = f - yk[o];
      loss += wk * e * e * scale;
      double df = act ? f * (1.0 - f) : (z3[o] > 0 ? 1.0 : 0.0);
      d3[o] = 2.0 * wk * e * scale * df;
    }
    if (!grad) continue;
    for (int i = 0; i < h2; ++i) {
      double s = 0;
      for (int o = 0; o < out; ++o) s += W3[(size_t)o * h2 + i] * d3[o];
      d2[i] = z2[i] > 0 ? s : 0.0;
    }
    for (int i = 0; i < h1; ++i) {
      double s = 0;
      for (int o = 0; o < h2; ++o) s += W2[(size_t)o * h1 + i] * d2[o];
      d1[i] = z1[i] > 0 ? s : 0.0;
    }
    for (int o = 0; o < out; ++o) {
      gb3[o] += d3[o];
      for (int i = 0; i < h2; ++i) gW3[(size_t)o * h2 + i] += d3[o] * (z2[i] > 0 ? z2[i] : 0.0);
    }
    for (int o = 0; o < h2; ++o) {
      gb2[o] += d2[o];
      for (int i = 0; i < h1; ++i) gW2[(size_t)o * h1 + i] += d2[o] * (z1[i] > 0 ? z1[i] : 0.0);
    }
    for (int o = 0; o < h1; ++o) {
      gb1[o] += d1[o];
      for (int i = 0; i < in; ++i) gW1[(size_t)o * in + i] += d1[o] * xk[i];
    }
  }
  free(z1);
  return loss;
}

double orc_mlp_loss_grad_act(const int32_t* dims, const double* w, const double* x, const double* y, int64_t B,
                             int32_t act, double* grad) {
  return orc_mlp_loss_grad_wt(dims, w, x, y, NULL, B, act, grad);
}

double orc_mlp_loss_grad(const int32_t* dims, const double* w, const double* x, const double* y, int64_t B,
                         double* grad) {
  return orc_mlp_loss_grad_act(dims, w, x, y, B, 0, grad);
}

/*
 * Adam (Kingma and Ba 2015), bias-corrected, step t >= 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 */
void orc_adam(int64_t n, double* w, double* m, double* v, const double* g, double lr, double b1, double b2,
              double eps, int32_t t) {
  double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    w[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------ */
/* Approximate baselines of the evaluation (Sec. 4): weighted blended OIT and  */
/* the naive renderer that blends in submission order with no OIT.             */

/*
 * WBOIT weight (McGuire and Bavoil, JCGT 2013), the variant driven by the
 * window-space depth z in [0,1] that the fragment lists carry:
 *   w(z, a) = a * max(1e-2, 3e3 * (1 - z)^3).
 * Reading: the evaluation names the authors' recommended weight without
 * giving it; of their published weights this is the one defined on the depth
 * buffer value, which is the depth the fragment lists hold.
 */
double orc_wboit_weight(double z, double a) {
  double u = 1.0 - z;
  double g = 3e3 * u * u * u;
  if (g < 1e-2) g = 1e-2;
  return a * g;
}

/*
 * method 0, WBOIT: over each list, in any order,
 *   acc = sum w_j a_j c_j,  wa = sum w_j a_j,  R = prod (1 - a_j)  (revealage),
 *   C = (acc / wa) (1 - R) + R C_b, with acc / wa = 0 when wa = 0.
 * method 1, submission-order over: eq (1) applied to each list as stored
 * (primitive order), without sorting: the paper's "random order" renderer.
 * rgb [P][3]. Returns 0, or -1 for an unknown method.
 */
int orc_baseline(int32_t W, int32_t H, const uint32_t* off, const float* depth, const float* rgba, int32_t method,
                 const double* bg, double* rgb) {
  int64_t P = (int64_t)W * H;
  if (method != 0 && method != 1) return -1;
  for (int64_t p = 0; p < P; ++p) {
    double C[3] = {0, 0, 0}, T = 1.0;
    if (method == 0) {
      double acc[3] = {0, 0, 0}, wa = 0.0;
      for (uint32_t i = off[p]; i < off[p + 1]; ++i) {
        double a = rgba[4 * (size_t)i + 3];
        double w = orc_wboit_weight(depth[i], a);
        for (int c = 0; c < 3; ++c) acc[c] += w * a * rgba[4 * (size_t)i + c];
        wa += w * a;
        T *= 1.0 - a;
      }
      for (int c = 0; c < 3; ++c) C[c] = wa > 0 ? acc[c] / wa * (1.0 - T) : 0.0;
    } else {
      for (uint32_t i = off[p]; i < off[p + 1]; ++i) {
        double a = rgba[4 * (size_t)i + 3];
        for (int c = 0; c < 3; ++c) C[c] += T * a * rgba[4 * (size_t)i + c];
        T *= 1.0 - a;
      }
    }
    for (int c = 0; c < 3; ++c) rgb[3 * p + c] = C[c] + T * bg[c];
  }
  return 0;
}
