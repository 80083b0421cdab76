"""Python binding of libstarnt.so: the MI355X (gfx950) per-pixel hot path of
STAR-NT neural order-independent transparency (arXiv 2606.16747).

Argument marshalling only: torch tensors provide device memory and the stream;
every step runs in the library's HIP kernels. The functions carry the C names
(starnt_features, starnt_infer, starnt_composite, starnt_quadtree,
starnt_reproject, starnt_train_step) and raise StarntError on a non-zero
status. The library must be built (`python -m paper_2606_16747_amd.build` or
__graft_entry__.build()); importing without it fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstarnt.so")

F32, F16, BF16, FP8 = 0, 1, 2, 3
MODE_LEARNED, MODE_F0, MODE_FAVG, MODE_EXACT = 0, 1, 2, 3
NET_STARNT, NET_DFAOIT = 0, 1
BASE_WBOIT, BASE_OVER_LIST = 0, 1
WS_QUADTREE, WS_TRAIN, WS_REPROJECT = 1, 2, 3
DERR_DEPTH, DERR_ALPHA, DERR_COUNT, DERR_LIST = 1, 2, 4, 8
STATUS = {0: "OK", 1: "EINVAL", 2: "ERANGE", 3: "ENOMEM", 4: "EHIP", 5: "EUNSUPPORTED"}
EINVAL, ERANGE, ENOMEM, EHIP, EUNSUPPORTED = 1, 2, 3, 4, 5

_P = ctypes.c_void_p


class StarntError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Frags(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("offsets", _P), ("depth", _P),
                ("rgba", _P), ("rgba_dtype", ctypes.c_int32), ("prim", _P), ("num_frags", ctypes.c_uint64),
                ("max_per_pixel", ctypes.c_uint32)]


class Sched(ctypes.Structure):
    _fields_ = [("w2", ctypes.c_int32), ("h2", ctypes.c_int32), ("w3", ctypes.c_int32), ("h3", ctypes.c_int32),
                ("hist", ctypes.c_uint32 * 4), ("wbar", ctypes.c_float), ("s2", ctypes.c_float),
                ("s3", ctypes.c_float), ("frames", ctypes.c_uint32), ("pad", ctypes.c_uint32 * 4)]


class Feats(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("d1", _P), ("layer1", _P),
                ("count", _P), ("layer2", _P), ("tail", _P), ("sel", _P), ("err", _P), ("tail_avg", _P)]


class Mlp(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_int32), ("h1", ctypes.c_int32), ("h2", ctypes.c_int32), ("out", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("W1", _P), ("b1", _P), ("W2", _P), ("b2", _P), ("W3", _P), ("b3", _P),
                ("fp8_scales", ctypes.POINTER(ctypes.c_float)), ("variant", ctypes.c_int32)]


class QtParams(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int32), ("tau_split", ctypes.c_float), ("tau_merge", ctypes.c_float),
                ("k_relax", ctypes.c_int32)]


class Train(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_int32), ("h1", ctypes.c_int32), ("h2", ctypes.c_int32), ("out", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("params", _P), ("m", _P), ("v", _P), ("grad", _P),
                ("out_act", ctypes.c_int32), ("weight", _P), ("fp8_act_scale", ctypes.c_float * 3)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int32)]


class Interval(ctypes.Structure):
    _fields_ = [("target_ms", ctypes.c_double), ("smoothing", ctypes.c_double), ("real_ms", ctypes.c_double),
                ("interp_ms", ctypes.c_double), ("max_interval", ctypes.c_int32), ("interval", ctypes.c_int32),
                ("pos", ctypes.c_int32), ("pad", ctypes.c_int32)]


assert ctypes.sizeof(Sched) == 64

EXPORTS = ("starnt_features", "starnt_infer", "starnt_infer_composite", "starnt_composite", "starnt_baseline",
           "starnt_dfa_inputs", "starnt_infer_composite_sel",
           "starnt_quadtree", "starnt_quadtree_noalloc", "starnt_reproject", "starnt_reproject_check", "starnt_patch", "starnt_interval_init", "starnt_interval_next",
           "starnt_interval_report",
           "starnt_train_step", "starnt_sched_init", "starnt_wbar", "starnt_pass_scales", "starnt_grid_dim",
           "starnt_workspace_size", "starnt_check", "starnt_last_error", "starnt_version", "starnt_m_minus_i",
           "starnt_time_next_launch")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libstarnt.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    lib.starnt_features.argtypes = [ctypes.POINTER(Frags), _P, ctypes.POINTER(Feats), _P]
    lib.starnt_infer.argtypes = [ctypes.POINTER(Mlp), _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]
    lib.starnt_infer_composite.argtypes = [ctypes.POINTER(Mlp), ctypes.POINTER(Feats), _P,
                                           ctypes.POINTER(ctypes.c_float), _P, _P]
    lib.starnt_composite.argtypes = [ctypes.POINTER(Frags), ctypes.POINTER(Feats), _P, _P,
                                     ctypes.POINTER(ctypes.c_float), ctypes.c_int32, _P, _P, _P]
    lib.starnt_dfa_inputs.argtypes = [ctypes.POINTER(Feats), _P, _P, _P]
    lib.starnt_infer_composite_sel.argtypes = [ctypes.POINTER(Mlp), ctypes.POINTER(Feats), _P, _P, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_float), _P, _P]
    lib.starnt_baseline.argtypes = [ctypes.POINTER(Frags), ctypes.c_int32, ctypes.POINTER(ctypes.c_float), _P, _P]
    lib.starnt_interval_init.argtypes = [ctypes.POINTER(Interval), ctypes.c_double, ctypes.c_int32, ctypes.c_double]
    lib.starnt_interval_next.argtypes = [ctypes.POINTER(Interval)]
    lib.starnt_interval_report.argtypes = [ctypes.POINTER(Interval), ctypes.c_int32, ctypes.c_double]
    lib.starnt_quadtree.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(QtParams), _P, _P, _P,
                                    _P, _P, ctypes.c_size_t, _P]
    lib.starnt_quadtree_noalloc.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(QtParams), _P,
                                            _P, _P, _P, _P]
    lib.starnt_reproject.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), _P,
                                     _P, _P]
    lib.starnt_reproject_check.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                           ctypes.c_float, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    lib.starnt_patch.argtypes = [ctypes.POINTER(Frags), ctypes.POINTER(Mlp), _P, _P, ctypes.POINTER(Feats),
                                 ctypes.POINTER(ctypes.c_float), _P, _P]
    lib.starnt_train_step.argtypes = [ctypes.POINTER(Train), _P, _P, ctypes.c_int32, ctypes.POINTER(Adam), _P, _P,
                                      ctypes.c_size_t, _P]
    lib.starnt_sched_init.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P]
    lib.starnt_wbar.restype = ctypes.c_double
    lib.starnt_wbar.argtypes = [ctypes.POINTER(ctypes.c_uint32)]
    lib.starnt_pass_scales.restype = None
    lib.starnt_pass_scales.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
    lib.starnt_grid_dim.restype = ctypes.c_int32
    lib.starnt_grid_dim.argtypes = [ctypes.c_int32, ctypes.c_double]
    lib.starnt_workspace_size.restype = ctypes.c_size_t
    lib.starnt_m_minus_i.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_float)]
    lib.starnt_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
    lib.starnt_check.argtypes = [ctypes.c_uint32]
    lib.starnt_time_next_launch.argtypes = [_P, _P]
    lib.starnt_last_error.restype = ctypes.c_char_p
    lib.starnt_version.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(rc):
    if rc != 0:
        raise StarntError(rc, lib.starnt_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    return t


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, device):
    return torch.as_tensor(t).to(device=device, dtype=dtype).contiguous()


# ---------------------------------------------------------------------------
# device-side containers (torch tensors) and their C views

class DeviceFrags:
    """A frame's fragment lists in device memory (see starnt_frags)."""

    def __init__(self, offsets, depth, rgba, prim, width, height, max_per_pixel, device="cuda"):
        self.width, self.height = int(width), int(height)
        self.offsets = _dev(np.asarray(offsets).view(np.int32), torch.int32, device)
        self.depth = _dev(depth, torch.float32, device)
        rgba = np.asarray(rgba)
        if rgba.dtype == np.float16:
            self.rgba = torch.from_numpy(rgba.view(np.int16)).to(device).contiguous()
            self.rgba_dtype = F16
        else:
            self.rgba = _dev(rgba, torch.float32, device)
            self.rgba_dtype = F32
        self.prim = _dev(np.asarray(prim).view(np.int32), torch.int32, device)
        self.num_frags = int(self.depth.shape[0])
        self.max_per_pixel = int(max_per_pixel)
        self._c = self.c()

    @classmethod
    def from_frame(cls, fr, max_per_pixel=None, device="cuda"):
        mx = int(max_per_pixel or max(1, int(fr.stats.get("max_count", 1)), 1))
        return cls(fr.offsets, fr.depth, fr.rgba, fr.prim, fr.width, fr.height, mx, device)

    def c(self):
        return Frags(self.width, self.height, self.offsets.data_ptr(), self.depth.data_ptr(), self.rgba.data_ptr(),
                     self.rgba_dtype, self.prim.data_ptr(), self.num_frags, self.max_per_pixel)

    @property
    def bytes_streamed(self):
        """Algorithmic bytes of one full-resolution pass: offsets + depth + RGBA."""
        per = 8 if self.rgba_dtype == F16 else 16
        return 4 * (self.width * self.height + 1) + self.num_frags * (4 + per)


class FeatBuffers:
    """Outputs of starnt_features (full-resolution capacity)."""

    def __init__(self, width, height, device="cuda", with_sel=False, with_avg=False):
        P = int(width) * int(height)
        self.width, self.height = int(width), int(height)
        self.d1 = torch.empty(P, dtype=torch.float32, device=device)
        self.layer1 = torch.empty(P, 4, dtype=torch.float32, device=device)
        self.count = torch.empty(P, dtype=torch.int32, device=device)
        self.layer2 = torch.zeros(P, 4, dtype=torch.float32, device=device)
        self.tail = torch.zeros(P, 8, dtype=torch.float32, device=device)
        self.sel = torch.empty(P, 2, dtype=torch.int32, device=device) if with_sel else None
        self.err = torch.zeros(1, dtype=torch.int32, device=device)
        self.tail_avg = torch.zeros(P, 4, dtype=torch.float32, device=device) if with_avg else None
        self._c = self.c()

    def c(self):
        return Feats(self.width, self.height, self.d1.data_ptr(), self.layer1.data_ptr(), self.count.data_ptr(),
                     self.layer2.data_ptr(), self.tail.data_ptr(),
                     self.sel.data_ptr() if self.sel is not None else None, self.err.data_ptr(),
                     self.tail_avg.data_ptr() if self.tail_avg is not None else None)


def new_sched(width, height, s2=1.0, s3=1.0, device="cuda", stream=None):
    """A device schedule (64 bytes) initialised to the given pass scales."""
    t = torch.zeros(16, dtype=torch.int32, device=device)
    starnt_sched_init(t, width, height, s2, s3, stream)
    return t


def read_sched(t):
    """Host copy of a device schedule as a dict (synchronises)."""
    raw = t.detach().cpu().numpy().astype(np.int32)
    s = Sched.from_buffer_copy(raw.tobytes())
    return {"w2": s.w2, "h2": s.h2, "w3": s.w3, "h3": s.h3, "hist": list(s.hist), "wbar": s.wbar, "s2": s.s2,
            "s3": s.s3, "frames": s.frames}


class DeviceMlp:
    """FP32 master weights of the tail network on the device."""

    def __init__(self, Ws, bs, dtype=F32, fp8_scales=None, device="cuda", variant=NET_STARNT):
        self.Ws = [_dev(w, torch.float32, device) for w in Ws]
        self.bs = [_dev(b, torch.float32, device) for b in bs]
        self.dims = (self.Ws[0].shape[1], self.Ws[0].shape[0], self.Ws[1].shape[0], self.Ws[2].shape[0])
        self.variant = int(variant)
        self.set_dtype(dtype, fp8_scales)

    def set_dtype(self, dtype, fp8_scales=None):
        self.dtype = dtype
        self._scales = None if fp8_scales is None else (ctypes.c_float * 6)(*[float(v) for v in fp8_scales])
        W, b = self.Ws, self.bs
        self._c = Mlp(self.dims[0], self.dims[1], self.dims[2], self.dims[3], dtype, W[0].data_ptr(),
                      b[0].data_ptr(), W[1].data_ptr(), b[1].data_ptr(), W[2].data_ptr(), b[2].data_ptr(),
                      self._scales, self.variant)
        return self


# ---------------------------------------------------------------------------
# the C calls

# number of starnt_features launches issued by this process (lets a profiler's
# per-dispatch records be matched to a caller's own launches)
features_launches = 0


def starnt_features(frags: DeviceFrags, sched, feats: FeatBuffers, stream=None):
    global features_launches
    _check(lib.starnt_features(ctypes.byref(frags._c), _ptr(sched), ctypes.byref(feats._c), _stream(stream)))
    features_launches += 1


def _event_handle(ev):
    if ev is None:
        return None
    h = int(ev.cuda_event)
    if h == 0:
        raise ValueError("starnt_time_next_launch: record the event once before passing it (torch creates it then)")
    return ctypes.c_void_p(h)


def starnt_time_next_launch(start=None, stop=None):
    """The calling thread's next fragment-pass, network or exact-path kernel
    records these torch.cuda.Events with its own dispatch (both None clears
    the request)."""
    _check(lib.starnt_time_next_launch(_event_handle(start), _event_handle(stop)))


def starnt_infer(mlp: DeviceMlp, tail, count, sched, width, height, tail_rgb, stream=None):
    _check(lib.starnt_infer(ctypes.byref(mlp._c), _ptr(tail), _ptr(count), _ptr(sched), int(width), int(height),
                            _ptr(tail_rgb), _stream(stream)))


def starnt_infer_composite(mlp: DeviceMlp, feats: FeatBuffers, sched, bg, rgb, stream=None):
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check(lib.starnt_infer_composite(ctypes.byref(mlp._c), ctypes.byref(feats._c), _ptr(sched), bgc, _ptr(rgb),
                                      _stream(stream)))


def starnt_composite(frags, feats, tail_rgb, sched, bg, mode, rgb, fstar=None, stream=None):
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check(lib.starnt_composite(ctypes.byref(frags._c) if frags is not None else None,
                                ctypes.byref(feats._c) if feats is not None else None, _ptr(tail_rgb), _ptr(sched),
                                bgc, int(mode), _ptr(rgb), _ptr(fstar), _stream(stream)))


def starnt_infer_composite_sel(mlp: DeviceMlp, feats: FeatBuffers, sched, level, base, bg, rgb, stream=None):
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check(lib.starnt_infer_composite_sel(ctypes.byref(mlp._c), ctypes.byref(feats._c), _ptr(sched), _ptr(level),
                                          int(base), bgc, _ptr(rgb), _stream(stream)))


def starnt_dfa_inputs(feats: FeatBuffers, sched, x, stream=None):
    _check(lib.starnt_dfa_inputs(ctypes.byref(feats._c), _ptr(sched), _ptr(x), _stream(stream)))


def starnt_baseline(frags, method, bg, rgb, stream=None):
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check(lib.starnt_baseline(ctypes.byref(frags._c) if frags is not None else None, int(method), bgc, _ptr(rgb),
                               _stream(stream)))


def starnt_interval_init(target_ms, max_interval=4, smoothing=0.25) -> Interval:
    s = Interval()
    _check(lib.starnt_interval_init(ctypes.byref(s), float(target_ms), int(max_interval), float(smoothing)))
    return s


def starnt_interval_next(s: Interval) -> bool:
    """True when the next frame is a real render, False for an interpolated one."""
    r = lib.starnt_interval_next(ctypes.byref(s))
    if r < 0:
        raise StarntError(1, "starnt_interval_next: NULL state")
    return bool(r)


def starnt_interval_report(s: Interval, was_real, ms):
    _check(lib.starnt_interval_report(ctypes.byref(s), int(bool(was_real)), float(ms)))


def starnt_quadtree(rgb, count, width, height, params: QtParams, prev_mask, mask, level, sched, workspace,
                    stream=None):
    _check(lib.starnt_quadtree(_ptr(rgb), _ptr(count), int(width), int(height), ctypes.byref(params),
                               _ptr(prev_mask), _ptr(mask), _ptr(level), _ptr(sched), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream)))


def starnt_quadtree_noalloc(rgb, count, width, height, params: QtParams, prev_mask, mask, level, sched,
                            stream=None):
    _check(lib.starnt_quadtree_noalloc(_ptr(rgb), _ptr(count), int(width), int(height), ctypes.byref(params),
                                       _ptr(prev_mask), _ptr(mask), _ptr(level), _ptr(sched), _stream(stream)))


def starnt_reproject(rgb_prev, d1_prev, width, height, m_minus_i, rgb_out, src=None, stream=None):
    m = np.asarray(m_minus_i, np.float32).ravel()
    mc = (ctypes.c_float * 16)(*[float(v) for v in m])
    _check(lib.starnt_reproject(_ptr(rgb_prev), _ptr(d1_prev), int(width), int(height), mc, _ptr(rgb_out), _ptr(src),
                                _stream(stream)))


def starnt_reproject_check(rgb_prev, d1_prev, width, height, m_minus_i, depth_tol, rgb_out, src, lst, count,
                           workspace, stream=None):
    """workspace: starnt_workspace_size(WS_REPROJECT, width, height) bytes."""
    m = np.asarray(m_minus_i, np.float32).ravel()
    mc = (ctypes.c_float * 16)(*[float(v) for v in m])
    _check(lib.starnt_reproject_check(_ptr(rgb_prev), _ptr(d1_prev), int(width), int(height), mc, float(depth_tol),
                                      _ptr(rgb_out), _ptr(src), _ptr(lst), _ptr(count), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream(stream)))


def starnt_patch(frags, mlp: DeviceMlp, lst, count, slots: FeatBuffers, bg, rgb, stream=None):
    """slots: FeatBuffers(capacity, 1), scratch for the listed pixels."""
    bgc = (ctypes.c_float * 3)(*[float(v) for v in bg])
    _check(lib.starnt_patch(ctypes.byref(frags._c) if frags is not None else None, ctypes.byref(mlp._c), _ptr(lst),
                            _ptr(count), ctypes.byref(slots._c) if slots is not None else None, bgc, _ptr(rgb),
                            _stream(stream)))


def starnt_train_step(train: Train, x, y, batch, adam: Adam, loss, workspace, stream=None):
    _check(lib.starnt_train_step(ctypes.byref(train), _ptr(x), _ptr(y), int(batch), ctypes.byref(adam), _ptr(loss),
                                 _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)))


def starnt_sched_init(sched, width, height, s2, s3, stream=None):
    _check(lib.starnt_sched_init(_ptr(sched), int(width), int(height), float(s2), float(s3), _stream(stream)))


def starnt_m_minus_i(vp_prev, vp_cur):
    """M - I, M = vp_prev vp_cur^-1, as float32[4, 4] (computed by the library)."""
    a = (ctypes.c_double * 16)(*[float(v) for v in np.asarray(vp_prev, np.float64).ravel()])
    b = (ctypes.c_double * 16)(*[float(v) for v in np.asarray(vp_cur, np.float64).ravel()])
    out = (ctypes.c_float * 16)()
    _check(lib.starnt_m_minus_i(a, b, out))
    return np.array(out, np.float32).reshape(4, 4)


def starnt_wbar(hist4):
    h = (ctypes.c_uint32 * 4)(*[int(v) for v in hist4])
    return float(lib.starnt_wbar(h))


def starnt_pass_scales(wbar):
    a, b = ctypes.c_double(), ctypes.c_double()
    lib.starnt_pass_scales(float(wbar), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def starnt_grid_dim(n, s):
    return int(lib.starnt_grid_dim(int(n), float(s)))


def starnt_workspace_size(kind, a, b, c=0):
    return int(lib.starnt_workspace_size(int(kind), int(a), int(b), int(c)))


def starnt_check(err_word):
    _check(lib.starnt_check(int(err_word) & 0xFFFFFFFF))


def starnt_version():
    return lib.starnt_version().decode()


def workspace(nbytes, device="cuda"):
    return torch.empty(max(1, (int(nbytes) + 255) // 256 * 256), dtype=torch.uint8, device=device)
