"""Kernel timing through starnt_time_next_launch: the fragment pass, the
network and the exact path record the caller's events with their own
dispatch. The timed call gives bitwise the same outputs as the untimed one,
its kernel time is positive and lies inside events recorded around the call,
and the request holds for one launch only."""
import numpy as np
import pytest
import torch

from gpu_util import sync, to_np

pytestmark = pytest.mark.gpu


def _events(n):
    """Timing events created up front (torch creates an event at its first
    record), as the library needs them."""
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    for e in evs:
        e.record()
    sync()
    return evs


def _frame(sg):
    return sg.Scene("c2_1080p", width=480, height=270, num_tris=300).frame(0)


def _timed(starnt, fn):
    """(kernel ms from the library's events, ms of events around the call)"""
    k0, k1, o0, o1 = _events(4)
    o0.record()
    starnt.starnt_time_next_launch(k0, k1)
    fn()
    o1.record()
    sync()
    return k0.elapsed_time(k1), o0.elapsed_time(o1)


def test_features_timed(starnt, sg, gpu):
    fr = _frame(sg)
    df = starnt.DeviceFrags.from_frame(fr)
    fa = starnt.FeatBuffers(fr.width, fr.height)
    fb = starnt.FeatBuffers(fr.width, fr.height)
    starnt.starnt_features(df, None, fa)
    k, o = _timed(starnt, lambda: starnt.starnt_features(df, None, fb))
    assert 0.0 < k <= o
    for name in ("d1", "layer1", "count", "layer2", "tail"):
        assert np.array_equal(to_np(getattr(fa, name)).view(np.uint32), to_np(getattr(fb, name)).view(np.uint32)), name


def test_exact_and_network_timed(starnt, sg, gpu):
    fr = _frame(sg)
    df = starnt.DeviceFrags.from_frame(fr)
    P = fr.width * fr.height
    ra = torch.empty(P, 3, dtype=torch.float32, device=gpu)
    rb = torch.empty(P, 3, dtype=torch.float32, device=gpu)
    starnt.starnt_composite(df, None, None, None, (1, 1, 1), starnt.MODE_EXACT, ra)
    k, o = _timed(starnt, lambda: starnt.starnt_composite(df, None, None, None, (1, 1, 1), starnt.MODE_EXACT, rb))
    assert 0.0 < k <= o
    assert np.array_equal(to_np(ra).view(np.uint32), to_np(rb).view(np.uint32))

    fb = starnt.FeatBuffers(fr.width, fr.height)
    starnt.starnt_features(df, None, fb)
    rng = np.random.default_rng(7)
    Ws = [rng.normal(0, 0.3, (32, 16)), rng.normal(0, 0.2, (32, 32)), rng.normal(0, 0.2, (3, 32))]
    bs = [rng.normal(0, 0.1, 32), rng.normal(0, 0.1, 32), np.full(3, 0.05)]
    mlp = starnt.DeviceMlp(Ws, bs, starnt.BF16)
    starnt.starnt_infer_composite(mlp, fb, None, (1, 1, 1), ra)
    k, o = _timed(starnt, lambda: starnt.starnt_infer_composite(mlp, fb, None, (1, 1, 1), rb))
    assert 0.0 < k <= o
    assert np.array_equal(to_np(ra).view(np.uint32), to_np(rb).view(np.uint32))


def test_request_is_one_shot(starnt, sg, gpu):
    """The second launch after a request leaves the events where the first
    one put them."""
    fr = _frame(sg)
    df = starnt.DeviceFrags.from_frame(fr)
    fb = starnt.FeatBuffers(fr.width, fr.height)
    k0, k1 = _events(2)
    starnt.starnt_time_next_launch(k0, k1)
    starnt.starnt_features(df, None, fb)
    sync()
    first = k0.elapsed_time(k1)
    starnt.starnt_features(df, None, fb)
    sync()
    assert k0.elapsed_time(k1) == first
    # both NULL clears a pending request
    starnt.starnt_time_next_launch(k0, k1)
    starnt.starnt_time_next_launch(None, None)
    starnt.starnt_features(df, None, fb)
    sync()
    assert k0.elapsed_time(k1) == first


def test_unrecorded_event_rejected(starnt, gpu):
    with pytest.raises(ValueError):
        starnt.starnt_time_next_launch(torch.cuda.Event(enable_timing=True), None)
