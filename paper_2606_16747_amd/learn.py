"""Training driver for the tail-colour network (Sec. 3.3: MSE, Adam).

Pairs (x, f*) come from the library itself: starnt_features gives the five
features at full resolution and the exact A-buffer path gives the exact tail
colour f* of every pixel with at least three fragments. For the DFAOIT
network the input is starnt_dfa_inputs and the target the whole transparent
colour C_t (the exact composite over a black background). Every gradient step
is starnt_train_step.

Loss weights: eq (3) adds T2 f to the composite, so an error e in f costs
T2 e in the image; weighting each sample's squared error by T2^2 trains on
the composite's own error (pixels whose tail is hidden behind two nearly
opaque layers count for little). The features pass writes each sample's T2
into its tail record.

Input scaling: each input is multiplied by a power of two for training (the
count N spans hundreds, the other features [0, 1]); the scale is folded into
layer 1 afterwards, so inference sees raw features. A power-of-two scale is
exact under bf16 and e4m3 rounding, so the narrow-operand products at
inference are bit for bit those of training.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (BF16, FP8, NET_DFAOIT, WS_TRAIN, Adam, DeviceFrags, FeatBuffers, Train,
               starnt_dfa_inputs, starnt_features, starnt_train_step, starnt_workspace_size, workspace)
from .frames import exact_frame


def pairs_from(frags: DeviceFrags, bg=(1.0, 1.0, 1.0), with_t2=False):
    """(x [M, 16], f* [M, 3]) on the host for the pixels with N >= 3, and
    their T2 [M] (from the tail records) when with_t2."""
    fb = FeatBuffers(frags.width, frags.height)
    starnt_features(frags, None, fb)
    P = frags.width * frags.height
    rgb = torch.empty(P, 3, dtype=torch.float32, device=fb.d1.device)
    fstar = torch.empty(P, 3, dtype=torch.float32, device=fb.d1.device)
    exact_frame(frags, rgb, bg, fstar)
    torch.cuda.synchronize()
    n = fb.count.cpu().numpy()
    keep = n >= 3
    rec = fb.tail.cpu().numpy()[keep]
    x = np.zeros((int(keep.sum()), 16), np.float32)
    x[:, :5] = rec[:, :5]
    if with_t2:
        return x, fstar.cpu().numpy()[keep], rec[:, 6].copy()
    return x, fstar.cpu().numpy()[keep]


def dfa_pairs_from(frags: DeviceFrags):
    """(x [M, 16], C_t [M, 3]) on the host for the pixels with N >= 3: the
    DFAOIT input and the exact transparent colour without background."""
    fb = FeatBuffers(frags.width, frags.height, with_avg=True)
    starnt_features(frags, None, fb)
    P = frags.width * frags.height
    x = torch.empty(P, 16, dtype=torch.float32, device=fb.d1.device)
    starnt_dfa_inputs(fb, None, x)
    ct = torch.empty(P, 3, dtype=torch.float32, device=fb.d1.device)
    exact_frame(frags, ct, (0.0, 0.0, 0.0))
    torch.cuda.synchronize()
    keep = fb.count.cpu().numpy() >= 3
    return x.cpu().numpy()[keep], ct.cpu().numpy()[keep]


class Pow2Scaler:
    """Per-input power-of-two scales 2^-k with 2^k the input's largest
    magnitude rounded up to a power of two (1 for inputs in [0, 1])."""

    def __init__(self, x, n_in=5):
        self.sc = np.ones(16)
        amax = np.abs(x[:, :n_in]).max(0)
        self.sc[:n_in] = np.exp2(-np.ceil(np.log2(np.maximum(amax, 1.0))))

    def apply(self, x):
        return (x * self.sc).astype(np.float32)

    def fold(self, W1, b1):
        """Layer 1 on raw x equal to layer 1 on scaled x (exact: the scales
        are powers of two)."""
        return (W1 * self.sc[None, :]).astype(np.float32), np.asarray(b1, np.float32)


def e4m3_scale(amax):
    """Smallest power of two s with amax / s <= 448 (1 for amax = 0): the
    rule the training kernel applies to each layer's weights."""
    amax = float(amax)
    if not amax > 0.0:
        return 1.0
    m, e = np.frexp(amax)  # amax = m 2^e, m in [0.5, 1); 448 = 0.875 2^9
    return float(np.ldexp(1.0, int(e) - 9 if m <= 0.875 else int(e) - 8))


def activation_amax(Ws, bs, x):
    """Largest magnitude of each layer's input over the samples x (FP64
    forward of the current weights), for the E4M3 activation scales."""
    amax = [float(np.abs(x).max())]
    h = np.asarray(x, np.float64)
    for w, b in list(zip(Ws, bs))[:2]:
        h = np.maximum(h @ np.asarray(w, np.float64).T + b, 0.0)
        amax.append(float(np.abs(h).max()))
    return amax


def fp8_inference_scales(Ws, bs, x):
    """The six scales (s_a, s_w per layer, powers of two) of an FP8 network
    for inputs like x: twice the observed activation range, the weights'."""
    sa = [e4m3_scale(2.0 * v) for v in activation_amax(Ws, bs, x)]
    sw = [e4m3_scale(np.abs(w).max()) for w in Ws]
    return [v for pair in zip(sa, sw) for v in pair]


def train(x, y, Ws, bs, steps=3000, batch=65536, lr=2e-3, lr_min=1e-4, dtype=BF16, seed=0, log_every=0,
          device="cuda", stream=None, variant=0, weight=None, fp8_every=250):
    """Train from initial weights (Ws, bs); returns (Ws, bs, losses) with the
    input scaling folded into layer 1. variant NET_DFAOIT trains the
    sigmoid-output network on its eleven inputs; weight [M] gives per-sample
    loss weights (None: plain MSE). dtype FP8 runs the forward products on
    E4M3 operands; the activation scales (twice the observed range, powers of
    two) are recalibrated from the current weights every fp8_every steps."""
    dims = (Ws[0].shape[1], Ws[0].shape[0], Ws[1].shape[0], Ws[2].shape[0])
    dfa = variant == NET_DFAOIT
    st = Pow2Scaler(x, 11 if dfa else 5)
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(x))
    xs = torch.from_numpy(st.apply(x[order])).to(device)
    ys = torch.from_numpy(np.ascontiguousarray(y[order], np.float32)).to(device)
    wts = None if weight is None else torch.from_numpy(np.ascontiguousarray(weight[order], np.float32)).to(device)
    M = len(x)
    batch = min(batch, M)
    nb = M // batch
    flat = np.concatenate([np.concatenate([np.asarray(w, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                           for w, b in zip(Ws, bs)])
    p = torch.from_numpy(flat).to(device)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.zeros_like(p)
    tr = Train(16, dims[1], dims[2], 3, dtype, p.data_ptr(), m.data_ptr(), v.data_ptr(), g.data_ptr(),
               1 if dfa else 0)
    ws = workspace(starnt_workspace_size(WS_TRAIN, batch, dims[1], dims[2]), device)
    loss = torch.zeros(steps, dtype=torch.float32, device=device)
    cal = st.apply(x[order[: min(len(x), 65536)]]).astype(np.float64)
    shapes = [(dims[1], dims[0]), (dims[1],), (dims[2], dims[1]), (dims[2],), (dims[3], dims[2]), (dims[3],)]

    def unflatten(flat_np):
        parts, k = [], 0
        for sh in shapes:
            n = int(np.prod(sh))
            parts.append(flat_np[k:k + n].reshape(sh))
            k += n
        return parts
    for t in range(steps):
        if dtype == FP8 and t % fp8_every == 0:
            parts = unflatten(p.cpu().numpy())
            amax = activation_amax(parts[0::2], parts[1::2], cal)
            for l in range(3):
                tr.fp8_act_scale[l] = e4m3_scale(2.0 * amax[l])
        b = int(rng.integers(nb))
        lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * t / max(1, steps)))
        ad = Adam(lr_t, 0.9, 0.999, 1e-8, t + 1)
        xb = xs[b * batch:(b + 1) * batch]
        yb = ys[b * batch:(b + 1) * batch]
        if wts is not None:
            tr.weight = wts[b * batch:(b + 1) * batch].data_ptr()
        starnt_train_step(tr, xb, yb, batch, ad, loss[t:t + 1], ws, stream)
        if log_every and (t % log_every == 0 or t == steps - 1):
            torch.cuda.synchronize()
            print("step %d loss %.3e" % (t, float(loss[t])), flush=True)
    torch.cuda.synchronize()
    parts = unflatten(p.cpu().numpy())
    W1, b1 = st.fold(parts[0].astype(np.float64), parts[1].astype(np.float64))
    return [W1, parts[2], parts[4]], [b1, parts[3], parts[5]], loss.cpu().numpy()
