"""Seeded synthetic transparent scenes as per-pixel fragment lists (CSR).

Input generation only: this package holds none of the compositing method's
arithmetic. Both the CPU oracle (tests) and the GPU library consume the arrays
it returns. Random numbers come from SplitMix64 streams keyed by
(seed, stream, index), so every frame is reproducible on its own.

CSR layout of one frame with P = width*height pixels and F fragments:
  offsets uint32[P+1]   pixel p owns fragments offsets[p] .. offsets[p+1]-1
  depth   float32[F]    NDC depth in [0, 1]
  rgba    float32[F,4]  straight (non-premultiplied) colour and opacity
                        (float16[F,4] when the scene asks for half RGBA)
  prim    uint32[F]     primitive id, unique within a pixel's list
Pixels are row-major (p = y*width + x), y = 0 the top row.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scenegen.cpp")
_LIB = os.path.join(_HERE, "_scenegen.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator with the host compiler (no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("num_tris", ctypes.c_int32), ("num_moving", ctypes.c_int32), ("num_frames", ctypes.c_int32),
        ("max_per_pixel", ctypes.c_uint32), ("shuffle", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("alpha_lo", ctypes.c_double), ("alpha_hi", ctypes.c_double),
        ("size_mu", ctypes.c_double), ("size_sigma", ctypes.c_double),
        ("clusters", ctypes.c_int32), ("cluster_frac", ctypes.c_double), ("cluster_radius", ctypes.c_double),
        ("depth_lo", ctypes.c_double), ("depth_hi", ctypes.c_double),
        ("fov_y_deg", ctypes.c_double), ("z_near", ctypes.c_double), ("z_far", ctypes.c_double),
        ("cam_rot_deg", ctypes.c_double), ("cam_trans", ctypes.c_double),
        ("move_rot_deg", ctypes.c_double), ("move_trans", ctypes.c_double),
        ("colour_mode", ctypes.c_int32), ("half_rgba", ctypes.c_int32),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("num_frags", ctypes.c_uint64), ("trimmed", ctypes.c_uint64), ("max_count", ctypes.c_uint32),
        ("mean_count", ctypes.c_double), ("p99_count", ctypes.c_uint32),
        ("covered_pixels", ctypes.c_uint32), ("dropped_tris", ctypes.c_uint32),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            lib.sg_create.restype = ctypes.c_void_p
            lib.sg_create.argtypes = [ctypes.POINTER(_Params)]
            lib.sg_destroy.argtypes = [ctypes.c_void_p]
            lib.sg_rasterize.restype = ctypes.c_int64
            lib.sg_rasterize.argtypes = [ctypes.c_void_p, ctypes.c_int32]
            lib.sg_fetch.restype = ctypes.c_int32
            lib.sg_fetch.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5 + [ctypes.POINTER(_Stats)]
            lib.sg_camera.restype = ctypes.c_int32
            lib.sg_camera.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
            lib.sg_uniform.restype = None
            lib.sg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
            _lib = lib
    return _lib


@dataclasses.dataclass
class SceneParams:
    kind: int = 0                 # 0 screen-space triangles, 1 world space + camera path
    width: int = 256
    height: int = 256
    num_tris: int = 64
    num_moving: int = 0
    num_frames: int = 1
    max_per_pixel: int = 0        # 0 = unlimited
    shuffle: bool = False
    seed: int = 0x57A20001
    alpha_lo: float = 0.2
    alpha_hi: float = 0.8
    size_mu: float = -2.0
    size_sigma: float = 0.6
    clusters: int = 0
    cluster_frac: float = 0.0
    cluster_radius: float = 0.05
    depth_lo: float = 4.0
    depth_hi: float = 20.0
    fov_y_deg: float = 60.0
    z_near: float = 0.5
    z_far: float = 50.0
    cam_rot_deg: float = 0.5
    cam_trans: float = 0.02
    move_rot_deg: float = 0.0
    move_trans: float = 0.0
    colour_mode: int = 0          # 0 iid colours, 1 correlated with depth, 2 per-object palette
    half_rgba: bool = False

    def _c(self) -> _Params:
        d = dataclasses.asdict(self)
        d["shuffle"] = int(d["shuffle"])
        d["half_rgba"] = int(d["half_rgba"])
        return _Params(**d)


BASE_SEED = 0x57A20000

# Synthetic workloads: sizes, depth-complexity targets and motion of the five
# measured configurations; the comment of each preset gives its statistics.
PRESETS = {
    # 256x256, 64 screen-space triangles, planar depth U[0,1], mean ~4-5, max ~24
    "c1_256": SceneParams(kind=0, width=256, height=256, num_tris=64, max_per_pixel=24,
                          seed=BASE_SEED + 1),
    # 1920x1080, 2000 world triangles, heavy-tailed (mean ~8, max 64), 8-frame
    # smooth camera path (<= 0.25 deg and 0.01 units per frame), per-object materials
    "c2_1080p": SceneParams(kind=1, width=1920, height=1080, num_tris=2000, num_frames=8,
                            max_per_pixel=64, seed=BASE_SEED + 2, size_mu=-2.03, size_sigma=0.55,
                            clusters=5, cluster_frac=0.5, cluster_radius=0.012,
                            cam_rot_deg=0.25, cam_trans=0.01, colour_mode=2),
    # 512x512 training scenes, mean ~12, max 128, per-object materials
    "c3_512": SceneParams(kind=1, width=512, height=512, num_tris=1600, max_per_pixel=128,
                          seed=BASE_SEED + 3, size_mu=-2.0, size_sigma=0.6,
                          clusters=2, cluster_frac=0.5, cluster_radius=0.002, colour_mode=2),
    # 3840x2160, 8000 triangles, mean ~16, max 256, fp16 RGBA
    "c4_4k": SceneParams(kind=1, width=3840, height=2160, num_tris=8000, max_per_pixel=256,
                         seed=BASE_SEED + 4, size_mu=-2.5, size_sigma=0.6, clusters=6,
                         cluster_frac=0.5, cluster_radius=0.004, half_rgba=True, colour_mode=2),
    # 2560x1440, 4000 static + 500 moving triangles, 60 frames, mean ~10, max 160
    "c5_1440p": SceneParams(kind=1, width=2560, height=1440, num_tris=4000, num_moving=500,
                            num_frames=60, max_per_pixel=160, seed=BASE_SEED + 5,
                            size_mu=-2.45, size_sigma=0.6, clusters=4, cluster_frac=0.5,
                            cluster_radius=0.005, cam_rot_deg=0.3, cam_trans=0.01,
                            move_rot_deg=0.5, move_trans=0.01, colour_mode=2),
}


@dataclasses.dataclass
class Frame:
    width: int
    height: int
    offsets: np.ndarray   # uint32[P+1]
    depth: np.ndarray     # float32[F]
    rgba: np.ndarray      # float32[F,4] or float16[F,4]
    prim: np.ndarray      # uint32[F]
    vp: np.ndarray        # float64[4,4] view-projection (row-major, column vectors)
    stats: dict

    @property
    def num_pixels(self) -> int:
        return self.width * self.height

    @property
    def num_frags(self) -> int:
        return int(self.depth.shape[0])

    def counts(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64)).astype(np.uint32)


class Scene:
    """A seeded scene: fixed triangles plus a camera path; frames on demand."""

    def __init__(self, params: SceneParams | str, **overrides):
        if isinstance(params, str):
            params = dataclasses.replace(PRESETS[params])
        if overrides:
            params = dataclasses.replace(params, **overrides)
        self.params = params
        self._lib = _load()
        self._cp = params._c()
        self._h = self._lib.sg_create(ctypes.byref(self._cp))
        if not self._h:
            raise ValueError("scenegen: invalid scene parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.sg_destroy(h)
            self._h = None

    def camera(self, frame: int) -> np.ndarray:
        vp = np.zeros(16, np.float64)
        if self._lib.sg_camera(self._h, int(frame), vp.ctypes.data) != 0:
            raise ValueError("scenegen: bad frame")
        return vp.reshape(4, 4)

    def frame(self, t: int = 0) -> Frame:
        W, H = self.params.width, self.params.height
        F = self._lib.sg_rasterize(self._h, int(t))
        if F < 0:
            raise ValueError("scenegen: rasterisation failed")
        offsets = np.empty(W * H + 1, np.uint32)
        depth = np.empty(F, np.float32)
        rgba = np.empty((F, 4), np.float32)
        prim = np.empty(F, np.uint32)
        vp = np.empty(16, np.float64)
        st = _Stats()
        rc = self._lib.sg_fetch(self._h, offsets.ctypes.data, depth.ctypes.data, rgba.ctypes.data,
                                prim.ctypes.data, vp.ctypes.data, ctypes.byref(st))
        if rc != 0:
            raise RuntimeError("scenegen: fetch failed")
        if self.params.half_rgba:
            rgba = rgba.astype(np.float16)
        stats = {k: getattr(st, k) for k, _ in _Stats._fields_}
        return Frame(W, H, offsets, depth, rgba, prim, vp.reshape(4, 4), stats)


def uniform(seed: int, stream: int, n: int, lo: float, hi: float) -> np.ndarray:
    """Seeded U[lo, hi) doubles (SplitMix64), e.g. for initial network weights."""
    out = np.empty(int(n), np.float64)
    _load().sg_uniform(int(seed), int(stream), int(n), float(lo), float(hi), out.ctypes.data)
    return out


def init_mlp(dims, seed: int = BASE_SEED + 100, out_bias: float = 0.0):
    """He-uniform weights W_l[out][in] (float32) and zero biases for an MLP with
    layer widths dims = (in, h1, h2, out). Returned as plain input data."""
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        lim = np.sqrt(6.0 / fan_in)
        w = uniform(seed, 10 + l, fan_in * fan_out, -lim, lim).astype(np.float32).reshape(fan_out, fan_in)
        Ws.append(w)
        b = np.zeros(fan_out, np.float32)
        if l == len(dims) - 2:
            b[:] = out_bias
        bs.append(b)
    return Ws, bs


def shuffled(frame: Frame, seed: int) -> Frame:
    """The same frame with every pixel's list permuted by a seeded shuffle."""
    rng = np.random.default_rng(seed)
    P = frame.num_pixels
    counts = frame.counts().astype(np.int64)
    pix = np.repeat(np.arange(P, dtype=np.int64), counts)
    key = rng.random(frame.num_frags)
    order = np.lexsort((key, pix))
    return Frame(frame.width, frame.height, frame.offsets.copy(), frame.depth[order].copy(),
                 frame.rgba[order].copy(), frame.prim[order].copy(), frame.vp.copy(), dict(frame.stats))
