"""FP64 CPU oracle for the STAR-NT per-pixel path (arXiv 2606.16747).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product library. It shares no code
with the GPU path; the plain C in oracle.c is the definition of every
quantity, written out with loops in double precision.

Parity pins (closed forms, invariants, brute force, finite differences) are in
tests/test_oracle_*.py. Functions without such a pin say so in their
docstring ("parity unpinned").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lock = threading.Lock()
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_P = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (plain C, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Mlp(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_int32), ("h1", ctypes.c_int32), ("h2", ctypes.c_int32),
                ("out", ctypes.c_int32)] + [(n, _P) for n in ("W1", "b1", "W2", "b2", "W3", "b3")]


class _QtParams(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int32), ("tau_split", ctypes.c_double), ("tau_merge", ctypes.c_double),
                ("k_relax", ctypes.c_int32)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            lib.orc_frame.restype = ctypes.c_int
            lib.orc_frame.argtypes = [ctypes.c_int32, ctypes.c_int32] + [_P] * 11 + [ctypes.c_int32]
            lib.orc_mlp_forward.restype = ctypes.c_int
            lib.orc_mlp_forward.argtypes = [ctypes.POINTER(_Mlp), _P, ctypes.c_int64, _P]
            lib.orc_mlp_forward_act.restype = ctypes.c_int
            lib.orc_mlp_forward_act.argtypes = [ctypes.POINTER(_Mlp), _P, ctypes.c_int64, ctypes.c_int32, _P]
            lib.orc_mlp_forward_q_act.restype = ctypes.c_int
            lib.orc_mlp_forward_q_amb.restype = ctypes.c_int
            lib.orc_mlp_forward_q_amb.argtypes = [ctypes.POINTER(_Mlp), _P, ctypes.c_int64, ctypes.c_int32, _P, _P,
                                                  ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P, _P, _P]
            lib.orc_mlp_forward_q_act.argtypes = [ctypes.POINTER(_Mlp), _P, ctypes.c_int64, ctypes.c_int32, _P, _P,
                                                  ctypes.c_int32, _P]
            lib.orc_mlp_loss_grad_act.restype = ctypes.c_double
            lib.orc_mlp_loss_grad_wt.restype = ctypes.c_double
            lib.orc_mlp_loss_grad_wt.argtypes = [_P, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32, _P]
            lib.orc_mlp_loss_grad_act.argtypes = [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32, _P]
            lib.orc_mlp_forward_q.restype = ctypes.c_int
            lib.orc_mlp_forward_q.argtypes = [ctypes.POINTER(_Mlp), _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P]
            lib.orc_round_bf16.restype = ctypes.c_double
            lib.orc_round_bf16.argtypes = [ctypes.c_double]
            lib.orc_round_e4m3.restype = ctypes.c_double
            lib.orc_round_e4m3.argtypes = [ctypes.c_double]
            lib.orc_grid_dim.restype = ctypes.c_int32
            lib.orc_grid_dim.argtypes = [ctypes.c_int32, ctypes.c_double]
            lib.orc_sample_pos.restype = ctypes.c_int32
            lib.orc_sample_pos.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
            lib.orc_upsample.restype = ctypes.c_int
            lib.orc_upsample.argtypes = [ctypes.c_int32] * 5 + [_P, _P]
            lib.orc_learned.restype = ctypes.c_int
            lib.orc_learned.argtypes = ([ctypes.c_int32] * 2 + [_P] * 2 + [ctypes.c_int32] * 4 +
                                        [ctypes.POINTER(_Mlp), ctypes.c_int32, _P, _P, _P, _P])
            lib.orc_wbar.restype = ctypes.c_double
            lib.orc_wbar.argtypes = [_P]
            lib.orc_pass_scales.restype = None
            lib.orc_pass_scales.argtypes = [ctypes.c_double, _D, _D]
            lib.orc_quadtree.restype = ctypes.c_int
            lib.orc_quadtree.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.POINTER(_QtParams),
                                         _P, _P, _P, _P, _P, _P]
            lib.orc_reproject.restype = ctypes.c_int
            lib.orc_reproject.argtypes = [ctypes.c_int32, ctypes.c_int32] + [_P] * 6
            lib.orc_reproject_full.restype = ctypes.c_int
            lib.orc_reproject_full.argtypes = [ctypes.c_int32, ctypes.c_int32] + [_P] * 5
            lib.orc_reproject_check.restype = ctypes.c_int
            lib.orc_reproject_check.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_double, _P, _P]
            lib.orc_inverse4.restype = ctypes.c_int
            lib.orc_inverse4.argtypes = [_P, _P]
            lib.orc_mlp_loss_grad.restype = ctypes.c_double
            lib.orc_mlp_loss_grad.argtypes = [_P, _P, _P, _P, ctypes.c_int64, _P]
            lib.orc_adam.restype = None
            lib.orc_adam.argtypes = [ctypes.c_int64, _P, _P, _P, _P, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int32]
            lib.orc_wboit_weight.restype = ctypes.c_double
            lib.orc_wboit_weight.argtypes = [ctypes.c_double, ctypes.c_double]
            lib.orc_baseline.restype = ctypes.c_int
            lib.orc_baseline.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.c_int32, _P, _P]
            _lib = lib
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------------------
# per-pixel exact quantities

def frame(offsets, depth, rgba, prim, width, height, bg=(1.0, 1.0, 1.0), nthreads=0, want=("rgb", "fstar", "lay", "tail", "sel")):
    """Exact A-buffer quantities of one frame (eq (1); Sec. 3.3 tail statistics).

    Returns a dict with (as requested):
      rgb   [P,3] exact composite over bg
      fstar [P,3] exact tail colour (sorted positions 3..N composited alone)
      lay   [P,10] N, d1, a1, c1(3), a2, c2(3)
      tail  [P,6] A, S(3), t_tail, 0
      sel   [P,2] global fragment index of layers 1 and 2 (0xFFFFFFFF if none)
      tavg  [P,4] tail means: colour sum c / (N-2) and opacity sum a / (N-2)
    """
    lib = _load()
    P = int(width) * int(height)
    off = _c(offsets, np.uint32)
    dep = _c(depth, np.float32)
    col = _c(np.asarray(rgba).astype(np.float32), np.float32)
    pr = _c(prim, np.uint32)
    bgv = np.asarray(bg, np.float64)
    out = {}
    bufs = {
        "rgb": np.empty((P, 3), np.float64) if "rgb" in want else None,
        "fstar": np.empty((P, 3), np.float64) if "fstar" in want else None,
        "lay": np.empty((P, 10), np.float64) if "lay" in want else None,
        "tail": np.empty((P, 6), np.float64) if "tail" in want else None,
        "sel": np.empty((P, 2), np.uint32) if "sel" in want else None,
        "tavg": np.empty((P, 4), np.float64) if "tavg" in want else None,
    }
    rc = lib.orc_frame(int(width), int(height), _ptr(off), _ptr(dep), _ptr(col), _ptr(pr), _ptr(bgv),
                       _ptr(bufs["rgb"]), _ptr(bufs["fstar"]), _ptr(bufs["lay"]), _ptr(bufs["tail"]),
                       _ptr(bufs["sel"]), _ptr(bufs["tavg"]), int(nthreads))
    if rc != 0:
        raise RuntimeError("orc_frame failed")
    for k, v in bufs.items():
        if v is not None:
            out[k] = v
    return out


def frame_of(fr, bg=(1.0, 1.0, 1.0), nthreads=0, want=("rgb", "fstar", "lay", "tail", "sel")):
    return frame(fr.offsets, fr.depth, fr.rgba, fr.prim, fr.width, fr.height, bg, nthreads, want)


def features(lay, tail):
    """[P,16] network input x = [N, t_tail, Ctilde_rgb, 0 x 11] (Sec. 3.3)."""
    P = lay.shape[0]
    x = np.zeros((P, 16), np.float64)
    A = tail[:, 0]
    x[:, 0] = lay[:, 0]
    x[:, 1] = tail[:, 4]
    with np.errstate(invalid="ignore", divide="ignore"):
        for c in range(3):
            x[:, 2 + c] = np.where(A > 0, tail[:, 1 + c] / np.where(A > 0, A, 1.0), 0.0)
    return x


# ---------------------------------------------------------------------------
# network

class Mlp:
    """Three dense layers W_l[out][in] (float32 data), ReLU after the hidden
    layers; the output activation is ReLU (act 0, STAR-NT) or the logistic
    sigmoid (act 1, the DFAOIT network)."""

    def __init__(self, Ws, bs, act=0):
        self.act = int(act)
        self.Ws = [np.ascontiguousarray(w, np.float32) for w in Ws]
        self.bs = [np.ascontiguousarray(b, np.float32) for b in bs]
        self.dims = (self.Ws[0].shape[1], self.Ws[0].shape[0], self.Ws[1].shape[0], self.Ws[2].shape[0])
        self._s = _Mlp(self.dims[0], self.dims[1], self.dims[2], self.dims[3],
                       *[a.ctypes.data for pair in zip(self.Ws, self.bs) for a in pair])

    def forward(self, x):
        x = _c(x, np.float64)
        n = x.shape[0]
        y = np.empty((n, self.dims[3]), np.float64)
        if _load().orc_mlp_forward_act(ctypes.byref(self._s), _ptr(x), n, self.act, _ptr(y)) != 0:
            raise RuntimeError("orc_mlp_forward failed")
        return y

    def forward_q(self, x, qmode, sa=None, sw=None):
        """Forward with narrow operands: qmode 1 = bf16, 2 = e4m3 with scales
        (pinned by hand-computed examples in test_oracle_pins_quant_mixed)."""
        x = _c(x, np.float64)
        n = x.shape[0]
        y = np.empty((n, self.dims[3]), np.float64)
        sa_ = _c(sa if sa is not None else np.ones(3), np.float64)
        sw_ = _c(sw if sw is not None else np.ones(3), np.float64)
        if _load().orc_mlp_forward_q_act(ctypes.byref(self._s), _ptr(x), n, int(qmode), _ptr(sa_), _ptr(sw_),
                                         self.act, _ptr(y)) != 0:
            raise RuntimeError("orc_mlp_forward_q failed")
        return y

    def forward_q_amb(self, x, qmode, sa=None, sw=None, tol_in=0.0, tol_h=0.0, with_mag=False):
        """forward_q plus, per sample, which rounded operands are ambiguous:
        bit 0 when an input moved by tol_in |v| rounds differently, bit 1 when
        a hidden activation moved by tol_h times the sum of the absolute terms
        (and bias) that produce it does. with_mag: also each output's sum of
        absolute terms and bias."""
        x = _c(x, np.float64)
        n = x.shape[0]
        y = np.empty((n, self.dims[3]), np.float64)
        amb = np.zeros(n, np.uint8)
        ym = np.empty((n, self.dims[3]), np.float64) if with_mag else None
        sa_ = _c(sa if sa is not None else np.ones(3), np.float64)
        sw_ = _c(sw if sw is not None else np.ones(3), np.float64)
        if _load().orc_mlp_forward_q_amb(ctypes.byref(self._s), _ptr(x), n, int(qmode), _ptr(sa_), _ptr(sw_),
                                         self.act, float(tol_in), float(tol_h), _ptr(y), _ptr(amb), _ptr(ym)) != 0:
            raise RuntimeError("orc_mlp_forward_q_amb failed")
        return (y, amb, ym) if with_mag else (y, amb)

    def params(self):
        """Flat FP64 parameter vector: W1, b1, W2, b2, W3, b3."""
        return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in zip(self.Ws, self.bs)]).astype(np.float64)


def round_bf16(v):
    lib = _load()
    return np.vectorize(lib.orc_round_bf16, otypes=[np.float64])(np.asarray(v, np.float64))


def round_e4m3(v):
    lib = _load()
    return np.vectorize(lib.orc_round_e4m3, otypes=[np.float64])(np.asarray(v, np.float64))


# ---------------------------------------------------------------------------
# mixed resolution, learned composite

def grid_dim(W, s):
    return int(_load().orc_grid_dim(int(W), float(s)))


def sample_pos(W, Ws, i):
    return int(_load().orc_sample_pos(int(W), int(Ws), int(i)))


def upsample(grid, W, H):
    """Bilinear upscale (half-pixel centres, clamp to edge) of [Hs,Ws,C] to [H,W,C]."""
    g = _c(grid, np.float64)
    Hs, Ws, C = g.shape
    out = np.empty((H, W, C), np.float64)
    _load().orc_upsample(int(W), int(H), int(Ws), int(Hs), int(C), _ptr(g), _ptr(out))
    return out


MODE_LEARNED, MODE_F0, MODE_FAVG = 0, 1, 2


def learned(lay, tail, width, height, grids, mlp: Mlp | None, mode=MODE_LEARNED, bg=(1.0, 1.0, 1.0)):
    """Learned-path composite (eq (3)) with passes 2/3 on the given grids
    (W2, H2, W3, H3). Returns (rgb [P,3], x [P,16], f [P,3])."""
    lib = _load()
    P = int(width) * int(height)
    W2, H2, W3, H3 = [int(v) for v in grids]
    rgb = np.empty((P, 3), np.float64)
    xf = np.empty((P, 16), np.float64)
    f = np.empty((P, 3), np.float64)
    bgv = np.asarray(bg, np.float64)
    if mode == MODE_LEARNED and mlp is None:
        raise ValueError("learned mode needs a network")
    ms = ctypes.byref(mlp._s) if mlp is not None else None
    rc = lib.orc_learned(int(width), int(height), _ptr(_c(lay, np.float64)), _ptr(_c(tail, np.float64)),
                         W2, H2, W3, H3, ms, int(mode), _ptr(bgv), _ptr(rgb), _ptr(xf), _ptr(f))
    if rc != 0:
        raise RuntimeError("orc_learned failed")
    return rgb, xf, f


# ---------------------------------------------------------------------------
# quadtree, pass scales

def wbar(hist4):
    h = _c(hist4, np.uint32)
    return float(_load().orc_wbar(_ptr(h)))


def pass_scales(wb):
    a, b = ctypes.c_double(), ctypes.c_double()
    _load().orc_pass_scales(float(wb), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def quadtree(rgb, N, width, height, base=64, tau_split=0.10, tau_merge=0.05, k_relax=2, prev_mask=None,
             force=None):
    """One quadtree update (Sec. 3.1). Returns (mask [T] u32, level [Ch,Cw] u8,
    hist [4] u32, D [T,21])."""
    lib = _load()
    W, H = int(width), int(height)
    Tw, Th = (W + base - 1) // base, (H + base - 1) // base
    cs = base // 8
    Cw, Ch = (W + cs - 1) // cs, (H + cs - 1) // cs
    rgbf = _c(np.asarray(rgb).reshape(-1, 3), np.float32)
    Nn = _c(N, np.uint32)
    mask = np.empty(Tw * Th, np.uint32)
    level = np.empty(Cw * Ch, np.uint8)
    hist = np.empty(4, np.uint32)
    D = np.empty((Tw * Th, 21), np.float64)
    pm = None if prev_mask is None else _c(prev_mask, np.uint32)
    fc = None if force is None else _c(force, np.int8)
    qp = _QtParams(int(base), float(tau_split), float(tau_merge), int(k_relax))
    rc = lib.orc_quadtree(W, H, _ptr(rgbf), _ptr(Nn), ctypes.byref(qp), _ptr(pm), _ptr(mask), _ptr(level),
                          _ptr(hist), _ptr(D), _ptr(fc))
    if rc != 0:
        raise RuntimeError("orc_quadtree failed")
    return mask, level.reshape(Ch, Cw), hist, D


# ---------------------------------------------------------------------------
# reprojection

def m_minus_i(vp_r, vp_t):
    """M - I with M = VP_r VP_t^-1, in FP64 (row-major, column vectors)."""
    inv = np.empty(16, np.float64)
    if _load().orc_inverse4(_ptr(_c(np.asarray(vp_t).ravel(), np.float64)), _ptr(inv)) != 0:
        raise ValueError("singular view-projection")
    M = np.asarray(vp_r, np.float64).reshape(4, 4) @ inv.reshape(4, 4)
    return M - np.eye(4)


def reproject(rgb_r, d1_r, mmi, width, height):
    """Gather of an interpolated frame from the last real frame (Sec. 3.3).
    Returns (rgb [P,3] float32, src [P] int32, margin [P] px to the nearest
    rounding boundary)."""
    W, H = int(width), int(height)
    P = W * H
    out = np.empty((P, 3), np.float32)
    src = np.empty(P, np.int32)
    mg = np.empty(P, np.float64)
    _load().orc_reproject(W, H, _ptr(_c(np.asarray(rgb_r).reshape(-1, 3), np.float32)),
                          _ptr(_c(d1_r, np.float32)), _ptr(_c(np.asarray(mmi).ravel(), np.float64)),
                          _ptr(out), _ptr(src), _ptr(mg))
    return out, src, mg


def reproject_full(d1_r, vp_r, vp_t, width, height):
    """Source pixel coordinates by explicit unprojection/projection."""
    W, H = int(width), int(height)
    su = np.empty(W * H, np.float64)
    sv = np.empty(W * H, np.float64)
    rc = _load().orc_reproject_full(W, H, _ptr(_c(d1_r, np.float32)), _ptr(_c(np.asarray(vp_r).ravel(), np.float64)),
                                    _ptr(_c(np.asarray(vp_t).ravel(), np.float64)), _ptr(su), _ptr(sv))
    if rc != 0:
        raise ValueError("singular view-projection")
    return su, sv


# ---------------------------------------------------------------------------
# training

def loss_grad(dims, params, x, y, act=0, wt=None):
    """MSE loss and its gradient for the flat parameter vector (FP64); act
    selects the output activation (0 ReLU, 1 sigmoid); wt the optional
    per-sample loss weights."""
    d = np.asarray(dims, np.int32)
    w = _c(params, np.float64)
    x = _c(x, np.float64)
    y = _c(y, np.float64)
    wt_ = _c(wt, np.float64) if wt is not None else None
    g = np.empty_like(w)
    loss = _load().orc_mlp_loss_grad_wt(_ptr(d), _ptr(w), _ptr(x), _ptr(y), _ptr(wt_), x.shape[0], int(act),
                                        _ptr(g))
    return loss, g


def adam(w, m, v, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, t=1):
    """In-place bias-corrected Adam step on FP64 arrays."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    _load().orc_adam(w.size, _ptr(w), _ptr(m), _ptr(v), _ptr(g), float(lr), float(b1), float(b2), float(eps), int(t))


def split_params(dims, flat):
    """Flat vector -> ([W1, W2, W3], [b1, b2, b3])."""
    i, h1, h2, o = dims
    shapes = [(h1, i), (h1,), (h2, h1), (h2,), (o, h2), (o,)]
    out, k = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(np.asarray(flat[k:k + n]).reshape(s))
        k += n
    return [out[0], out[2], out[4]], [out[1], out[3], out[5]]


# ---------------------------------------------------------------------------
# metrics

def psnr(a, b, mask=None):
    """10 log10(1 / MSE) over all channels (unclamped)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = (a - b) ** 2
    if mask is not None:
        d = d[np.asarray(mask)]
    mse = float(d.mean()) if d.size else 0.0
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


# ---------------------------------------------------------------------------
# approximate baselines of the evaluation (Sec. 4)

BASE_WBOIT = 0
BASE_OVER_LIST = 1


def wboit_weight(z, a):
    """McGuire-Bavoil weight on window-space depth: a * max(1e-2, 3e3 (1 - z)^3)."""
    return float(_load().orc_wboit_weight(float(z), float(a)))


def baseline(offsets, depth, rgba, width, height, method, bg=(1.0, 1.0, 1.0)):
    """[P,3] composite of a cheap baseline: method BASE_WBOIT (weighted blended
    OIT) or BASE_OVER_LIST (eq (1) in stored order, no sort)."""
    lib = _load()
    P = int(width) * int(height)
    off = _c(offsets, np.uint32)
    dep = _c(depth, np.float32)
    col = _c(np.asarray(rgba).astype(np.float32), np.float32)
    out = np.empty((P, 3), np.float64)
    rc = lib.orc_baseline(int(width), int(height), _ptr(off), _ptr(dep), _ptr(col), int(method),
                          _ptr(np.asarray(bg, np.float64)), _ptr(out))
    if rc != 0:
        raise ValueError("unknown baseline method %r" % (method,))
    return out


# ---------------------------------------------------------------------------
# adaptive interpolation interval (Sec. 3.3)

def interval_schedule(costs, target_ms, max_interval=4, smoothing=0.25):
    """Kinds of a sequence of frames under the adaptive interval: frames
    alternate one real render with (interval - 1) reprojected ones, the
    interval (at most max_interval <= 4) being re-chosen at every real frame
    from the running mean costs so the mean frame time meets target_ms with
    the least interpolation; a real frame that meets the target alone, or a
    target that even the longest interval misses, means every frame is real.
    Before any interpolated frame is measured, a real frame over the target
    is followed by one probing interval of two.

    Reading (the paper states the behaviour, not a rule): "meets" is mean
    time (real + (k-1) interp) / k <= target; running means move by
    smoothing * (sample - mean), starting at the first sample.

    costs[t] = (cost if frame t is real, cost if it is interpolated), in ms.
    Returns (kinds, means): kinds a list of booleans (True = real), means the
    final (real_ms, interp_ms), None where nothing was measured."""
    mean = {True: None, False: None}
    kinds = []
    interval, pos = 1, 0
    for t in range(len(costs)):
        if pos == 0:
            r, i = mean[True], mean[False]
            if r is None or r <= target_ms or max_interval < 2:
                interval = 1
            elif i is None:
                interval = 2
            else:
                interval = 1
                for k in range(2, max_interval + 1):
                    if (r + (k - 1) * i) / k <= target_ms:
                        interval = k
                        break
        real = pos == 0
        pos = (pos + 1) % interval
        kinds.append(real)
        c = costs[t][0 if real else 1]
        m = mean[real]
        mean[real] = c if m is None else m + smoothing * (c - m)
    return kinds, (mean[True], mean[False])


# ---------------------------------------------------------------------------
# the DFAOIT network's inputs and composite (Sec. 3.3, eq (2))

def dfa_features(lay, tail, tavg):
    """[P,16] DFAOIT input: the exact two-layer colour a1 c1 + (1-a1) a2 c2,
    the tail's mean colour and mean opacity, the tail's accumulated
    premultiplied colour C_acc = sum a c, and N; then zeros.
    Reading: the paper counts ten features for these items (eleven values);
    all listed items are used."""
    P = lay.shape[0]
    x = np.zeros((P, 16), np.float64)
    a1, c1, a2, c2 = lay[:, 2:3], lay[:, 3:6], lay[:, 6:7], lay[:, 7:10]
    x[:, 0:3] = a1 * c1 + (1.0 - a1) * a2 * c2
    x[:, 3:6] = tavg[:, 0:3]
    x[:, 6] = tavg[:, 3]
    x[:, 7:10] = tail[:, 1:4]
    x[:, 10] = lay[:, 0]
    return x


def dfa_composite(lay, tail, f, bg=(1.0, 1.0, 1.0)):
    """eq (2): C = C_t + C_b prod_i (1 - a_i) with C_t the network output where
    N >= 3 and the exact two-layer colour where N <= 2 (reading: both methods
    leave the tail-free pixels exact, so the ablation differs only where
    there is a tail)."""
    a1, c1, a2, c2 = lay[:, 2:3], lay[:, 3:6], lay[:, 6:7], lay[:, 7:10]
    exact2 = a1 * c1 + (1.0 - a1) * a2 * c2
    T = (1.0 - a1) * (1.0 - a2) * tail[:, 4:5]
    Ct = np.where(lay[:, 0:1] >= 3, f, exact2)
    return Ct + T * np.asarray(bg, np.float64)[None, :]


def dfa_learned(lay, tail, tavg, width, height, grids, mlp, bg=(1.0, 1.0, 1.0)):
    """The DFAOIT path with passes 2/3 on the given grids (W2, H2, W3, H3):
    layer 2 (a2, a2 c2) sampled on the pass-2 grid and the per-sample tail
    quantities (N, t_tail, S = sum a c, tail means) on the pass-3 grid are
    upscaled bilinearly (upsample), the full-resolution N gates them (no
    layer 2 where N < 2, no tail where N < 3), the input is dfa_features of
    the upscaled values, and eq (2) composites. mlp is None for the inputs
    alone. Returns (rgb [P,3], x [P,16], f [P,3]). Pinned at s < 1 by
    hand-computed upscale weights (test_oracle_pins_quant_mixed)."""
    W, H = int(width), int(height)
    P = W * H
    W2, H2, W3, H3 = [int(v) for v in grids]
    lay = np.asarray(lay, np.float64)
    tail = np.asarray(tail, np.float64)
    tavg = np.asarray(tavg, np.float64)
    g2 = np.zeros((H2, W2, 4))
    for j in range(H2):
        for i in range(W2):
            L = lay[sample_pos(H, H2, j) * W + sample_pos(W, W2, i)]
            g2[j, i] = (L[6], L[6] * L[7], L[6] * L[8], L[6] * L[9])
    g3 = np.zeros((H3, W3, 9))
    for j in range(H3):
        for i in range(W3):
            p = sample_pos(H, H3, j) * W + sample_pos(W, W3, i)
            g3[j, i] = (lay[p, 0], tail[p, 4], *tail[p, 1:4], *tavg[p])
    u2 = upsample(g2, W, H).reshape(P, 4)
    u3 = upsample(g3, W, H).reshape(P, 9)
    N = lay[:, 0]
    u2[N < 2] = 0.0
    a1, c1 = lay[:, 2:3], lay[:, 3:6]
    a2, pc2 = u2[:, 0:1], u2[:, 1:4]
    exact2 = a1 * c1 + (1.0 - a1) * pc2
    tailed = N >= 3
    x = np.zeros((P, 16))
    x[:, 0:3] = exact2
    x[:, 3:6] = u3[:, 5:8]
    x[:, 6] = u3[:, 8]
    x[:, 7:10] = u3[:, 2:5]
    x[:, 10] = u3[:, 0]
    x[~tailed] = 0.0
    f = np.zeros((P, 3))
    if mlp is not None and tailed.any():
        f[tailed] = mlp.forward(x[tailed])
    tt = np.where(tailed, u3[:, 1], 1.0)[:, None]
    Ct = np.where(tailed[:, None], f, exact2)
    rgb = Ct + (1.0 - a1) * (1.0 - a2) * tt * np.asarray(bg, np.float64)[None, :]
    return rgb, x, f


def selective(lay, tail, width, height, grids, mlp, level, base, bg=(1.0, 1.0, 1.0)):
    """Spatially selective inference: the learned composite (eq (3)), except
    that pixels whose quadtree cell (base / 8 px) is a level-0 leaf use the
    order-free tail f_avg. eq (3) is the same in both; only f differs."""
    W, H = int(width), int(height)
    rgb_l, _, _ = learned(lay, tail, W, H, grids, mlp, MODE_LEARNED, bg)
    rgb_a, _, _ = learned(lay, tail, W, H, grids, None, MODE_FAVG, bg)
    cs = int(base) // 8
    Cw = (W + cs - 1) // cs
    ys, xs = np.divmod(np.arange(W * H), W)
    flat = np.asarray(level).ravel()[(ys // cs) * Cw + xs // cs] == 0
    return np.where(flat[:, None], rgb_a, rgb_l)


def reproject_check(d1_r, mmi, width, height, tol):
    """Trust codes of the gather: q (trusted source), -2 (depth mismatch
    beyond tol), -1 (outside the frame or behind the camera); and the depth
    difference at the source."""
    W, H = int(width), int(height)
    code = np.empty(W * H, np.int32)
    zd = np.empty(W * H, np.float64)
    _load().orc_reproject_check(W, H, _ptr(_c(d1_r, np.float32)), _ptr(_c(np.asarray(mmi).ravel(), np.float64)),
                                float(tol), _ptr(code), _ptr(zd))
    return code, zd
