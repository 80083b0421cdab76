"""Frame scheduler of STAR-NT (Sec. 3, Fig. 1; interpolated frames Sec. 3.3).

A real frame runs passes 1-3 on the grids the device schedule holds, the tail
network, the eq (3) composite and the quadtree update, which leaves the next
frame's grids in the schedule (eq (4)); no host round trip is needed between
frames. An interpolated frame is one reprojection gather from the last real
frame; given that frame's fragment lists it also re-renders the pixels the
gather cannot trust (source outside the frame, behind the camera, or showing
another surface). Every step is a libstarnt call on the caller's stream.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (MODE_EXACT, MODE_LEARNED, WS_QUADTREE, WS_REPROJECT, DeviceFrags, DeviceMlp, FeatBuffers, QtParams,
               starnt_composite, starnt_features, starnt_infer_composite, starnt_infer_composite_sel,
               starnt_interval_init,
               starnt_interval_next, starnt_interval_report, starnt_m_minus_i, starnt_patch, starnt_quadtree,
               starnt_reproject,
               starnt_reproject_check, starnt_sched_init,
               starnt_workspace_size, workspace)


def m_minus_i(vp_real, vp_cur):
    """M - I with M = VP_real VP_cur^-1 (the library's host helper, FP64 then FP32)."""
    return starnt_m_minus_i(vp_real, vp_cur)


class Renderer:
    """Buffers and calls for one frame size. Outputs are [P, 3] float32.
    With selective=True a real frame after the first runs the network only
    off the flat (level-0) leaves of the last real frame's quadtree.
    depth_tol is the trust test's tolerance on window-space depth for
    interpolated frames that are given their fragment lists."""

    def __init__(self, width, height, mlp: DeviceMlp, base=64, tau_split=0.10, tau_merge=0.05, k_relax=2,
                 bg=(1.0, 1.0, 1.0), device="cuda", mode=MODE_LEARNED, selective=False, depth_tol=0.01):
        self.selective = bool(selective)
        self.depth_tol = float(depth_tol)
        self.W, self.H = int(width), int(height)
        P = self.W * self.H
        self.mlp = mlp
        self.mode = mode
        self.bg = tuple(float(v) for v in bg)
        self.qp = QtParams(int(base), float(tau_split), float(tau_merge), int(k_relax))
        self.feats = FeatBuffers(self.W, self.H, device)
        self.sched = torch.zeros(16, dtype=torch.int32, device=device)
        T = ((self.W + base - 1) // base) * ((self.H + base - 1) // base)
        cs = base // 8
        C = ((self.W + cs - 1) // cs) * ((self.H + cs - 1) // cs)
        self.masks = [torch.zeros(T, dtype=torch.int32, device=device) for _ in range(2)]
        self.level = torch.zeros(C, dtype=torch.uint8, device=device)
        self.ws = workspace(starnt_workspace_size(WS_QUADTREE, self.W, self.H, base), device)
        self.rgb_real = None
        self.n_real = 0
        # untrusted pixels of an interpolated frame and the slots of their
        # features (allocated on first use)
        self.list = torch.empty(P, dtype=torch.int32, device=device)
        self.list_count = torch.zeros(1, dtype=torch.int32, device=device)
        self.slots = None
        self.ws_reproj = workspace(starnt_workspace_size(WS_REPROJECT, self.W, self.H), device)
        self.device = device
        self.timer = None  # optional callable(name, fn) wrapping each call

    def _call(self, name, fn):
        if self.timer is None:
            fn()
        else:
            self.timer(name, fn)

    def reset(self, stream=None):
        """Start a sequence: full-resolution grids, no quadtree history."""
        starnt_sched_init(self.sched, self.W, self.H, 1.0, 1.0, stream)
        self.n_real = 0
        self.rgb_real = None

    def real_frame(self, frags: DeviceFrags, out, stream=None):
        self._call("features", lambda: starnt_features(frags, self.sched, self.feats, stream))
        if self.mode == MODE_LEARNED and self.selective and self.n_real > 0:
            self._call("infer_composite", lambda: starnt_infer_composite_sel(
                self.mlp, self.feats, self.sched, self.level, self.qp.base, self.bg, out, stream))
        elif self.mode == MODE_LEARNED:
            self._call("infer_composite", lambda: starnt_infer_composite(self.mlp, self.feats, self.sched, self.bg,
                                                                         out, stream))
        else:
            self._call("composite", lambda: starnt_composite(frags, self.feats, None, self.sched, self.bg,
                                                             self.mode, out, None, stream))
        prev = None if self.n_real == 0 else self.masks[(self.n_real - 1) % 2]
        cur = self.masks[self.n_real % 2]
        self._call("quadtree", lambda: starnt_quadtree(out, self.feats.count, self.W, self.H, self.qp, prev, cur,
                                                       self.level, self.sched, self.ws, stream))
        # feats.d1 keeps this frame's first-fragment depth until the next real
        # frame overwrites it, which stream order places after the gathers
        self.rgb_real = out
        self.n_real += 1
        return out

    def interpolated_frame(self, mmi, out, stream=None, frags: DeviceFrags | None = None):
        """The gather from the last real frame; with the frame's own fragment
        lists (learned mode), its untrusted pixels are rendered afresh."""
        assert self.rgb_real is not None, "an interpolated frame needs a real frame before it"
        if frags is None or self.mode != MODE_LEARNED:
            self._call("reproject", lambda: starnt_reproject(self.rgb_real, self.feats.d1, self.W, self.H, mmi, out,
                                                             None, stream))
            return out
        if self.slots is None:
            self.slots = FeatBuffers(self.W * self.H, 1, self.device)
        self._call("reproject", lambda: starnt_reproject_check(self.rgb_real, self.feats.d1, self.W, self.H, mmi,
                                                               self.depth_tol, out, None, self.list,
                                                               self.list_count, self.ws_reproj, stream))
        self._call("patch", lambda: starnt_patch(frags, self.mlp, self.list, self.list_count, self.slots, self.bg,
                                                 out, stream))
        return out


class AdaptiveSequence:
    """Frames of a sequence, each a real render or a reprojection of the last
    real frame, as the adaptive interval policy (starnt_interval_*) decides
    from measured frame costs (Sec. 3.3: at most four frames per real render,
    every frame real when the target is out of reach).

    Costs are measured with events around each frame and reported when the
    next frame is issued (one frame late, so the host never waits on the
    frame it just queued). `cost` may instead be a callable (t, real) -> ms
    that supplies them, which makes a sequence deterministic. The output of a
    real frame is the source of the frames interpolated after it, so it must
    stay untouched until the next real frame. With patch=True an interpolated
    frame also takes its fragment lists and re-renders its untrusted pixels."""

    def __init__(self, renderer: Renderer, target_ms, max_interval=4, smoothing=0.25, cost=None, patch=False):
        self.r = renderer
        self.patch = bool(patch)
        self.state = starnt_interval_init(target_ms, max_interval, smoothing)
        self.cost = cost
        self.vp_real = None
        self.t = 0
        self.kinds = []
        self._pending = None

    def _report(self):
        if self._pending is None:
            return
        t, real, a, b = self._pending
        if self.cost is not None:
            ms = float(self.cost(t, real))
        else:
            b.synchronize()
            ms = a.elapsed_time(b)
        starnt_interval_report(self.state, real, ms)
        self._pending = None

    def frame(self, vp, frags_fn, out, stream=None):
        """Render frame t into out; frags_fn() gives its fragment lists and is
        called only for a real frame (and, with patch, for every frame).
        Returns True for a real frame."""
        self._report()
        real = starnt_interval_next(self.state)
        if self.t == 0 or self.r.n_real == 0:
            assert real, "the first frame of a sequence is real"
        a = b = None
        if self.cost is None:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream) if stream is not None else a.record()
        if real:
            self.r.real_frame(frags_fn(), out, stream)
            self.vp_real = np.asarray(vp, np.float64)
        else:
            self.r.interpolated_frame(m_minus_i(self.vp_real, vp), out, stream,
                                      frags=frags_fn() if self.patch else None)
        if b is not None:
            b.record(stream) if stream is not None else b.record()
        self._pending = (self.t, real, a, b)
        self.kinds.append(real)
        self.t += 1
        return real


def exact_frame(frags: DeviceFrags, out, bg=(1.0, 1.0, 1.0), fstar=None, stream=None):
    starnt_composite(frags, None, None, None, bg, MODE_EXACT, out, fstar, stream)
    return out
