"""The DFAOIT variant (Sec. 3.3, eq (2)) on the GPU against the oracle: tail
means from the fragment pass, the upscaled ten-feature input, the FP32 and
BF16 composite with the sigmoid network, the sigmoid training step, and the
ten-versus-five-feature ablation after training both networks the same way."""
import numpy as np
import pytest
import torch

from gpu_util import run_exact, sync, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _grids(oracle_mod, W, H, s2, s3):
    return (oracle_mod.grid_dim(W, s2), oracle_mod.grid_dim(H, s2), oracle_mod.grid_dim(W, s3),
            oracle_mod.grid_dim(H, s3))


def _run(st, fr, s2, s3):
    W, H = fr.width, fr.height
    sched = st.new_sched(W, H, s2, s3)
    df = st.DeviceFrags.from_frame(fr, max_per_pixel=64)
    fb = st.FeatBuffers(W, H, with_avg=True)
    st.starnt_features(df, sched, fb)
    sync()
    return df, fb, sched


@pytest.mark.parametrize("s2,s3", [(1.0, 1.0), (0.5, 0.25), (0.77, 0.31)])
def test_tail_means_and_dfa_inputs(starnt, gpu, sg, oracle_mod, s2, s3):
    fr = sg.Scene("c1_256", width=250, height=131, num_tris=60).frame(0)
    W, H = fr.width, fr.height
    df, fb, sched = _run(starnt, fr, s2, s3)
    grids = _grids(oracle_mod, W, H, s2, s3)
    o = oracle_mod.frame_of(fr, want=("lay", "tail", "tavg"))
    # tail means at the pass-3 grid samples
    W3, H3 = grids[2], grids[3]
    ys = np.array([oracle_mod.sample_pos(H, H3, j) for j in range(H3)])
    xs = np.array([oracle_mod.sample_pos(W, W3, i) for i in range(W3)])
    pix = (ys[:, None] * W + xs[None, :]).ravel()
    ta = to_np(fb.tail_avg)[:W3 * H3]
    np.testing.assert_allclose(ta, o["tavg"][pix], rtol=0, atol=2e-6)
    # the upscaled input
    x = torch.empty(W * H, 16, dtype=torch.float32, device="cuda")
    starnt.starnt_dfa_inputs(fb, sched, x)
    sync()
    _, want, _ = oracle_mod.dfa_learned(o["lay"], o["tail"], o["tavg"], W, H, grids, None)
    got = to_np(x)
    np.testing.assert_allclose(got[:, :10], want[:, :10], rtol=0, atol=2e-5)
    np.testing.assert_allclose(got[:, 10], want[:, 10], rtol=1e-6, atol=2e-5)
    assert np.all(got[:, 11:] == 0)
    assert (o["lay"][:, 0] >= 3).sum() > 1000


@pytest.mark.parametrize("s2,s3", [(1.0, 1.0), (0.5, 0.25)])
def test_dfa_composite_fp32(starnt, gpu, sg, oracle_mod, s2, s3):
    fr = sg.Scene("c1_256", width=250, height=131, num_tris=60).frame(0)
    W, H = fr.width, fr.height
    df, fb, sched = _run(starnt, fr, s2, s3)
    Ws, bs = sg.init_mlp((16, 32, 32, 3), seed=61, out_bias=0.0)
    mlp = starnt.DeviceMlp(Ws, bs, starnt.F32, variant=starnt.NET_DFAOIT)
    rgb = torch.empty(W * H, 3, dtype=torch.float32, device="cuda")
    bg = (0.9, 0.2, 0.4)
    starnt.starnt_infer_composite(mlp, fb, sched, bg, rgb)
    sync()
    o = oracle_mod.frame_of(fr, want=("lay", "tail", "tavg"))
    want, _, _ = oracle_mod.dfa_learned(o["lay"], o["tail"], o["tavg"], W, H, _grids(oracle_mod, W, H, s2, s3),
                                        oracle_mod.Mlp(Ws, bs, act=1), bg=bg)
    assert np.abs(to_np(rgb) - want).max() <= TOL


def test_dfa_composite_bf16_against_same_operands(starnt, gpu, sg, oracle_mod):
    fr = sg.Scene("c1_256").frame(0)
    W, H = fr.width, fr.height
    df, fb, sched = _run(starnt, fr, 1.0, 1.0)
    Ws, bs = sg.init_mlp((16, 32, 32, 3), seed=62, out_bias=0.0)
    mlp = starnt.DeviceMlp(Ws, bs, starnt.BF16, variant=starnt.NET_DFAOIT)
    rgb = torch.empty(W * H, 3, dtype=torch.float32, device="cuda")
    starnt.starnt_infer_composite(mlp, fb, None, (1, 1, 1), rgb)
    sync()
    o = oracle_mod.frame_of(fr, want=("lay", "tail", "tavg"))
    x = oracle_mod.dfa_features(o["lay"], o["tail"], o["tavg"])
    tailed = o["lay"][:, 0] >= 3
    f = np.zeros((W * H, 3))
    f[tailed] = oracle_mod.Mlp(Ws, bs, act=1).forward_q(x[tailed], 1)
    want = oracle_mod.dfa_composite(o["lay"], o["tail"], f, (1, 1, 1))
    err = np.abs(to_np(rgb) - want).max(axis=1)
    assert np.mean(err <= 2e-4) >= 0.995, np.mean(err <= 2e-4)
    assert err.max() <= 2e-2


def test_train_step_sigmoid_fp32_gradient(starnt, gpu, sg, oracle_mod):
    fr = sg.Scene("c3_512", width=128, height=128, num_tris=200).frame(0)
    o = oracle_mod.frame_of(fr, want=("rgb", "lay", "tail", "tavg"))
    x = oracle_mod.dfa_features(o["lay"], o["tail"], o["tavg"])
    ct = oracle_mod.frame_of(fr, bg=(0, 0, 0), want=("rgb",))["rgb"]
    keep = o["lay"][:, 0] >= 3
    x, y = x[keep][:2000].astype(np.float32), ct[keep][:2000].astype(np.float32)
    x[:, 10] /= 16.0  # keep the sigmoid off saturation
    dims = (16, 32, 32, 3)
    Ws, bs = sg.init_mlp(dims, seed=63, out_bias=0.0)
    params = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in zip(Ws, bs)]).astype(np.float32)
    n = params.size
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    p, m, v, g = dev(params.copy()), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    tr = starnt.Train(16, 32, 32, 3, starnt.F32, p.data_ptr(), m.data_ptr(), v.data_ptr(), g.data_ptr(), 1)
    loss = torch.zeros(1, device="cuda")
    batch = len(x)
    ws = starnt.workspace(starnt.starnt_workspace_size(starnt.WS_TRAIN, batch, 32, 32))
    starnt.starnt_train_step(tr, dev(x), dev(y), batch, starnt.Adam(1e-3, 0.9, 0.999, 1e-8, 1), loss, ws)
    sync()
    lw, gw = oracle_mod.loss_grad(dims, params.astype(np.float64), x, y, act=1)
    gg = to_np(g).astype(np.float64)
    assert np.linalg.norm(gg - gw) / np.linalg.norm(gw) <= 1e-5
    assert abs(float(to_np(loss)[0]) - lw) <= 1e-5 * lw + 1e-9


def test_ablation_ten_versus_five_features(starnt, gpu, sg, capsys):
    """Both networks (16-32-32-3, BF16, same steps, batch and scenes) trained
    on 32 config-3 scenes and judged on 8 held-out ones at full resolution:
    STAR-NT (five features, tail colour, ReLU) and DFAOIT (ten features,
    whole colour, sigmoid). Stated, with the no-network f_avg for reference.
    STAR-NT must beat dropping the tail by 10 dB and DFAOIT by 5 dB (it
    predicts the exact two-layer part too, so its errors reach it; measured
    about 34 and 25 dB here)."""
    from paper_2606_16747_amd import learn
    xs5, ys5, xs10, ys10 = [], [], [], []
    for k in range(32):
        fr = sg.Scene("c3_512", seed=sg.BASE_SEED + 3 + 1000 * (k + 1)).frame(0)
        df = starnt.DeviceFrags.from_frame(fr, max_per_pixel=256)
        x, y = learn.pairs_from(df)
        xs5.append(x); ys5.append(y)
        x, y = learn.dfa_pairs_from(df)
        xs10.append(x); ys10.append(y)
    rng = np.random.default_rng(0)
    nets = {}
    for name, xs, ys, variant in (("starnt", xs5, ys5, starnt.NET_STARNT), ("dfaoit", xs10, ys10, starnt.NET_DFAOIT)):
        x, y = np.concatenate(xs), np.concatenate(ys)
        pick = rng.choice(len(x), min(len(x), 4_000_000), replace=False)
        Ws0, bs0 = sg.init_mlp((16, 32, 32, 3), seed=sg.BASE_SEED + 100, out_bias=0.05)
        Ws, bs, losses = learn.train(x[pick], y[pick], Ws0, bs0, steps=1500, lr=2e-3, batch=65536,
                                     dtype=starnt.BF16, variant=variant)
        nets[name] = (Ws, bs, losses)
    res = {"starnt": [], "dfaoit": [], "favg": [], "f0": []}
    for k in range(8):
        fr = sg.Scene("c3_512", seed=sg.BASE_SEED + 3 + 77777 * (k + 1)).frame(0)
        df = starnt.DeviceFrags.from_frame(fr, max_per_pixel=256)
        fb = starnt.FeatBuffers(fr.width, fr.height, with_avg=True)
        starnt.starnt_features(df, None, fb)
        exact, _ = run_exact(starnt, df)
        rgb = torch.empty(fr.num_pixels, 3, dtype=torch.float32, device="cuda")
        for name, variant in (("starnt", starnt.NET_STARNT), ("dfaoit", starnt.NET_DFAOIT)):
            Ws, bs, _ = nets[name]
            starnt.starnt_infer_composite(starnt.DeviceMlp(Ws, bs, starnt.BF16, variant=variant), fb, None,
                                          (1, 1, 1), rgb)
            sync()
            d = to_np(rgb).astype(np.float64) - exact
            res[name].append(10 * np.log10(1.0 / (d * d).mean()))
        for name, mode in (("favg", starnt.MODE_FAVG), ("f0", starnt.MODE_F0)):
            starnt.starnt_composite(df, fb, None, None, (1, 1, 1), mode, rgb)
            sync()
            d = to_np(rgb).astype(np.float64) - exact
            res[name].append(10 * np.log10(1.0 / (d * d).mean()))
    m = {k: float(np.mean(v)) for k, v in res.items()}
    with capsys.disabled():
        print("\n[ablation, config-3 held-out PSNR] STAR-NT 5 features %.2f dB, DFAOIT 10 features %.2f dB, "
              "f_avg %.2f, f=0 %.2f; final loss %.3e / %.3e" % (m["starnt"], m["dfaoit"], m["favg"], m["f0"],
                                                                  nets["starnt"][2][-20:].mean(),
                                                                  nets["dfaoit"][2][-20:].mean()))
    assert m["starnt"] > m["f0"] + 10.0
    assert m["dfaoit"] > m["f0"] + 5.0


def test_dfa_composite_fp8_against_same_operands(starnt, gpu, sg, oracle_mod):
    """FP8 (E4M3, per-layer scales) DFAOIT composite against the oracle on
    e4m3-rounded operands; the bar of the other FP8 tests (one e4m3 step per
    rounding flip), relative to the colour."""
    fr = sg.Scene("c1_256").frame(0)
    W, H = fr.width, fr.height
    df, fb, sched = _run(starnt, fr, 1.0, 1.0)
    o = oracle_mod.frame_of(fr, want=("lay", "tail", "tavg"))
    x = oracle_mod.dfa_features(o["lay"], o["tail"], o["tavg"])
    tailed = o["lay"][:, 0] >= 3
    Ws, bs = sg.init_mlp((16, 32, 32, 3), seed=64, out_bias=0.0)
    sa, sw = [], []
    h = x[tailed]
    for w, b in zip(Ws, bs):
        sa.append(float(np.abs(h).max()) / 448.0)
        sw.append(float(np.abs(w).max()) / 448.0)
        h = np.maximum(h @ w.T.astype(np.float64) + b, 0.0)
    mlp = starnt.DeviceMlp(Ws, bs, starnt.FP8, fp8_scales=[v for pair in zip(sa, sw) for v in pair],
                           variant=starnt.NET_DFAOIT)
    rgb = torch.empty(W * H, 3, dtype=torch.float32, device="cuda")
    starnt.starnt_infer_composite(mlp, fb, None, (1, 1, 1), rgb)
    sync()
    f = np.zeros((W * H, 3))
    f[tailed] = oracle_mod.Mlp(Ws, bs, act=1).forward_q(x[tailed], 2, np.array(sa), np.array(sw))
    want = oracle_mod.dfa_composite(o["lay"], o["tail"], f, (1, 1, 1))
    err = np.abs(to_np(rgb) - want).max(axis=1)
    assert np.mean(err <= 2e-3) >= 0.99, np.mean(err <= 2e-3)
    assert (err <= 0.25 * (np.abs(want).max(axis=1) + 0.1)).all(), err.max()


def test_tail_means_half_colour(starnt, gpu, sg, oracle_mod):
    """FP16 colour (the 4K workload's format) through the fragment pass with
    tail means: every pass-3 sample's means against the oracle."""
    fr = sg.Scene("c1_256", half_rgba=True, width=200, height=90, num_tris=50).frame(0)
    W, H = fr.width, fr.height
    df = starnt.DeviceFrags.from_frame(fr, max_per_pixel=64)
    assert df.rgba_dtype == starnt.F16
    sched = starnt.new_sched(W, H, 1.0, 0.6)
    fb = starnt.FeatBuffers(W, H, with_avg=True)
    starnt.starnt_features(df, sched, fb)
    sync()
    grids = _grids(oracle_mod, W, H, 1.0, 0.6)
    o = oracle_mod.frame_of(fr, want=("lay", "tail", "tavg"))
    W3, H3 = grids[2], grids[3]
    ys = np.array([oracle_mod.sample_pos(H, H3, j) for j in range(H3)])
    xs = np.array([oracle_mod.sample_pos(W, W3, i) for i in range(W3)])
    pix = (ys[:, None] * W + xs[None, :]).ravel()
    np.testing.assert_allclose(to_np(fb.tail_avg)[:W3 * H3], o["tavg"][pix], rtol=0, atol=2e-6)
    np.testing.assert_array_equal(to_np(fb.count).view(np.uint32), o["lay"][:, 0].astype(np.uint32))
    assert int(to_np(fb.err)[0]) == 0
