"""Parity of the cheap baselines (Sec. 4) with the FP64 oracle: weighted
blended OIT and blending in stored order, element by element on seeded frames
(several 64-pixel rows of quads and a ragged width), FP16 colour, long lists
and empty pixels. Bar: 2e-5 per channel (FP32 sums against FP64)."""
import numpy as np
import pytest
import torch

from csr_util import make_csr, random_lists
from gpu_util import sync, to_np

pytestmark = pytest.mark.gpu

TOL = 2e-5
BG = (0.25, 0.5, 0.75)


def _run(st, df, method, bg=BG):
    rgb = torch.empty(df.width * df.height, 3, dtype=torch.float32, device="cuda")
    st.starnt_baseline(df, method, bg, rgb)
    sync()
    return to_np(rgb)


@pytest.mark.parametrize("method", [0, 1])
def test_baseline_config1_frame(starnt, gpu, sg, oracle_mod, method):
    fr = sg.Scene("c1_256").frame(0)
    df = starnt.DeviceFrags.from_frame(fr)
    got = _run(starnt, df, method)
    want = oracle_mod.baseline(fr.offsets, fr.depth, fr.rgba, fr.width, fr.height, method, BG)
    np.testing.assert_allclose(got, want, rtol=0, atol=TOL)


@pytest.mark.parametrize("method", [0, 1])
def test_baseline_ragged_frame_random_lists(starnt, gpu, oracle_mod, method):
    rng = np.random.default_rng(11 + method)
    W, H = 37, 23
    lists = random_lists(rng, W, H, 30)
    off, dep, rgba, prim = make_csr(lists, W, H)
    df = starnt.DeviceFrags(off, dep, rgba, prim, W, H, 30)
    got = _run(starnt, df, method)
    want = oracle_mod.baseline(off, dep, rgba, W, H, method, BG)
    np.testing.assert_allclose(got, want, rtol=0, atol=TOL)


@pytest.mark.parametrize("method", [0, 1])
def test_baseline_half_colour(starnt, gpu, sg, oracle_mod, method):
    fr = sg.Scene("c1_256", half_rgba=True).frame(0)
    df = starnt.DeviceFrags.from_frame(fr)
    got = _run(starnt, df, method)
    want = oracle_mod.baseline(fr.offsets, fr.depth, fr.rgba.astype(np.float32), fr.width, fr.height, method, BG)
    np.testing.assert_allclose(got, want, rtol=0, atol=TOL)


@pytest.mark.parametrize("method", [0, 1])
def test_baseline_long_lists_and_empty_pixels(starnt, gpu, oracle_mod, method):
    """Lists of 0, 1, 3, 4, 5 and 3001 fragments side by side."""
    rng = np.random.default_rng(21)
    lists = []
    for n in (0, 1, 3, 4, 5, 3001, 0, 2):
        l = []
        for k in range(n):
            r, g, b = rng.random(3)
            l.append((float(rng.random()), k, float(r), float(g), float(b), float(rng.uniform(0.0, 0.05))))
        lists.append(l)
    off, dep, rgba, prim = make_csr(lists, 4, 2)
    df = starnt.DeviceFrags(off, dep, rgba, prim, 4, 2, 3001)
    got = _run(starnt, df, method)
    want = oracle_mod.baseline(off, dep, rgba, 4, 2, method, BG)
    np.testing.assert_allclose(got, want, rtol=0, atol=TOL)
    np.testing.assert_array_equal(got[0], np.float32(BG))


def test_over_list_on_sorted_lists_matches_exact_path(starnt, gpu, sg):
    """On lists stored front to back, blending in stored order is the exact
    path's result (both on the GPU)."""
    fr = sg.Scene("c1_256").frame(0)
    pix = np.repeat(np.arange(fr.num_pixels), fr.counts().astype(np.int64))
    order = np.lexsort((fr.prim, fr.depth, pix))  # per pixel by (depth, prim)
    df = starnt.DeviceFrags(fr.offsets, fr.depth[order], fr.rgba[order], fr.prim[order], fr.width, fr.height, 24)
    got = _run(starnt, df, 1)
    ex = torch.empty(fr.num_pixels, 3, dtype=torch.float32, device="cuda")
    starnt.starnt_composite(df, None, None, None, BG, starnt.MODE_EXACT, ex)
    sync()
    np.testing.assert_allclose(got, to_np(ex), rtol=0, atol=TOL)


@pytest.mark.parametrize("s2,s3", [(1.0, 1.0), (0.5, 0.31)])
def test_selective_inference_against_oracle(starnt, gpu, sg, oracle_mod, s2, s3):
    """Flat quadtree cells take f_avg, the rest the network (FP32), on a
    seeded level map; the same map is given to the oracle."""
    fr = sg.Scene("c1_256", width=250, height=131, num_tris=60).frame(0)
    W, H = fr.width, fr.height
    sched = starnt.new_sched(W, H, s2, s3)
    df = starnt.DeviceFrags.from_frame(fr, max_per_pixel=64)
    fb = starnt.FeatBuffers(W, H)
    starnt.starnt_features(df, sched, fb)
    base = 64
    Cw, Ch = (W + 7) // 8, (H + 7) // 8
    lv = np.random.default_rng(9).integers(0, 4, Cw * Ch).astype(np.uint8)
    Ws, bs = sg.init_mlp((16, 32, 32, 3), seed=65, out_bias=0.05)
    mlp = starnt.DeviceMlp(Ws, bs, starnt.F32)
    rgb = torch.empty(W * H, 3, dtype=torch.float32, device="cuda")
    starnt.starnt_infer_composite_sel(mlp, fb, sched, torch.from_numpy(lv).cuda(), base, BG, rgb)
    sync()
    o = oracle_mod.frame_of(fr, want=("lay", "tail"))
    grids = (oracle_mod.grid_dim(W, s2), oracle_mod.grid_dim(H, s2), oracle_mod.grid_dim(W, s3),
             oracle_mod.grid_dim(H, s3))
    want = oracle_mod.selective(o["lay"], o["tail"], W, H, grids, oracle_mod.Mlp(Ws, bs), lv, base, BG)
    assert np.abs(to_np(rgb) - want).max() <= 1e-4
    # BF16 on the matrix cores with the same mixed map: pixels off the flat
    # cells equal the fused BF16 call bit for bit (a column's network result
    # does not depend on its neighbours), flat pixels are the f_avg composite
    mlp.set_dtype(starnt.BF16)
    starnt.starnt_infer_composite_sel(mlp, fb, sched, torch.from_numpy(lv).cuda(), base, BG, rgb)
    full = torch.empty(W * H, 3, dtype=torch.float32, device="cuda")
    starnt.starnt_infer_composite(mlp, fb, sched, BG, full)
    sync()
    favg, _, _ = oracle_mod.learned(o["lay"], o["tail"], W, H, grids, None, oracle_mod.MODE_FAVG, BG)
    ys, xs = np.divmod(np.arange(W * H), W)
    flat = lv[(ys // 8) * Cw + xs // 8] == 0
    assert flat.any() and (~flat).any()
    np.testing.assert_array_equal(to_np(rgb)[~flat], to_np(full)[~flat])
    assert np.abs(to_np(rgb)[flat] - favg[flat]).max() <= 1e-4
    # an all-flat map runs no network at all
    starnt.starnt_infer_composite_sel(mlp, fb, sched, torch.from_numpy(np.zeros_like(lv)).cuda(), base, BG, rgb)
    sync()
    assert np.abs(to_np(rgb) - favg).max() <= 1e-4
