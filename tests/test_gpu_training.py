"""The learned part on the GPU: the network is trained by starnt_train_step on
(feature, exact tail colour) pairs produced by the library's own exact path,
and judged on held-out scenes against the exact compositor (Sec. 3.3: MSE,
Adam). Also: training state round-trips bitwise through a host checkpoint."""
import numpy as np
import pytest
import torch

from gpu_util import run_exact, sync, to_np

pytestmark = pytest.mark.gpu


def _held_out_psnr(st, sg, Ws, bs, seeds, mode, dtype=None, fp8_scales=None):
    """Mean PSNR of the full-resolution learned composite against the exact one."""
    out = []
    for s in seeds:
        fr = sg.Scene("c3_512", seed=s).frame(0)
        df = st.DeviceFrags.from_frame(fr, max_per_pixel=256)
        fb = st.FeatBuffers(fr.width, fr.height)
        st.starnt_features(df, None, fb)
        exact, _ = run_exact(st, df)
        rgb = torch.empty(fr.num_pixels, 3, dtype=torch.float32, device="cuda")
        if mode == "learned":
            kw = {"fp8_scales": fp8_scales} if fp8_scales is not None else {}
            mlp = st.DeviceMlp(Ws, bs, dtype if dtype is not None else st.F32, **kw)
            st.starnt_infer_composite(mlp, fb, None, (1, 1, 1), rgb)
        else:
            m = st.MODE_F0 if mode == "f0" else st.MODE_FAVG
            st.starnt_composite(df, fb, None, None, (1, 1, 1), m, rgb)
        sync()
        d = to_np(rgb).astype(np.float64) - exact
        out.append((10 * np.log10(1.0 / (d * d).mean()), np.abs(d).max()))
    return float(np.mean([p for p, _ in out])), float(max(m for _, m in out))


_C3 = {}


def _c3_pairs(starnt, sg):
    """The config-3 training pairs (32 seeded 512x512 scenes; at most 4M
    pairs) with each sample's T2, generated once per session."""
    if "pairs" not in _C3:
        from paper_2606_16747_amd import learn
        xs, ys, ts = [], [], []
        for k in range(32):
            fr = sg.Scene("c3_512", seed=sg.BASE_SEED + 3 + 1000 * (k + 1)).frame(0)
            x, y, t2 = learn.pairs_from(starnt.DeviceFrags.from_frame(fr, max_per_pixel=256), with_t2=True)
            xs.append(x)
            ys.append(y)
            ts.append(t2)
        x, y, t2 = np.concatenate(xs), np.concatenate(ys), np.concatenate(ts)
        pick = np.random.default_rng(0).choice(len(x), min(len(x), 4_000_000), replace=False)
        _C3["pairs"] = (x[pick], y[pick], t2[pick])
    return _C3["pairs"]


def test_fp8_training_held_out(starnt, gpu, sg, capsys):
    """16-64-64-3 trained with FP8 forward products (E4M3 operands, per-layer
    power-of-two scales) and FP32 masters on the config-3 pairs, evaluated
    with the FP8 network on the 8 held-out scenes: far better than dropping
    the tail and within 1.5 dB of the same training in BF16 (both stated)."""
    from paper_2606_16747_amd import learn
    x, y, t2 = _c3_pairs(starnt, sg)
    Ws0, bs0 = sg.init_mlp((16, 64, 64, 3), seed=sg.BASE_SEED + 100, out_bias=0.05)
    held = [sg.BASE_SEED + 3 + 77777 * (k + 1) for k in range(8)]
    res = {}
    for name, dt in (("fp8", starnt.FP8), ("bf16", starnt.BF16)):
        Ws, bs, losses = learn.train(x, y, Ws0, bs0, steps=1500, lr=2e-3, batch=65536, dtype=dt, weight=t2 ** 2)
        assert np.isfinite(losses).all() and losses[-20:].mean() < 0.25 * losses[:5].mean()
        if dt == starnt.FP8:
            sc = learn.fp8_inference_scales(Ws, bs, x[:65536].astype(np.float64))
            res[name] = _held_out_psnr(starnt, sg, Ws, bs, held, "learned", starnt.FP8, fp8_scales=sc)
        else:
            res[name] = _held_out_psnr(starnt, sg, Ws, bs, held, "learned", starnt.BF16)
    p_f0, _ = _held_out_psnr(starnt, sg, Ws0, bs0, held, "f0")
    with capsys.disabled():
        print("\n[FP8 training] held-out PSNR: FP8-trained, FP8 inference %.2f dB (max err %.3f); BF16-trained, "
              "BF16 inference %.2f dB; f=0 %.2f" % (res["fp8"][0], res["fp8"][1], res["bf16"][0], p_f0))
    assert res["fp8"][0] > p_f0 + 10.0
    assert res["fp8"][0] > res["bf16"][0] - 1.5


def test_config3_training_gain_over_no_network(starnt, gpu, sg, capsys):
    """32 training scenes (512x512, mean depth ~12), 16-64-64-3 in BF16 with
    FP32 masters, batch 65536, the T2^2-weighted loss. On 8 held-out scenes
    the trained network is far better than dropping the tail (f = 0) and than
    its untrained start, and within 1.5 dB of the order-free weighted-average
    tail f_avg: the five features carry no order, and f_avg is close to the
    mean tail colour given them, which bounds what any network on these
    features can reach (both numbers stated)."""
    from paper_2606_16747_amd import learn
    x, y, t2 = _c3_pairs(starnt, sg)
    Ws0, bs0 = sg.init_mlp((16, 64, 64, 3), seed=sg.BASE_SEED + 100, out_bias=0.05)
    Ws, bs, losses = learn.train(x, y, Ws0, bs0, steps=1500, lr=2e-3, batch=65536, dtype=starnt.BF16,
                                 weight=t2 ** 2)
    assert losses[-20:].mean() < 0.25 * losses[:5].mean()
    held = [sg.BASE_SEED + 3 + 77777 * (k + 1) for k in range(8)]
    p_learn, e_learn = _held_out_psnr(starnt, sg, Ws, bs, held, "learned", starnt.BF16)
    p_f32, _ = _held_out_psnr(starnt, sg, Ws, bs, held, "learned", starnt.F32)
    p_f0, _ = _held_out_psnr(starnt, sg, Ws, bs, held, "f0")
    p_favg, _ = _held_out_psnr(starnt, sg, Ws, bs, held, "favg")
    p_init, _ = _held_out_psnr(starnt, sg, Ws0, bs0, held, "learned", starnt.BF16)
    with capsys.disabled():
        print("\n[config-3 training] held-out PSNR: learned BF16 %.2f dB (FP32 network %.2f; max err %.3f), "
              "f=0 %.2f, f_avg %.2f, untrained %.2f; loss %.3e -> %.3e"
              % (p_learn, p_f32, e_learn, p_f0, p_favg, p_init, losses[:5].mean(), losses[-20:].mean()))
    assert p_learn > p_f0 + 10.0
    assert p_learn > p_init + 5.0
    assert abs(p_learn - p_favg) < 1.5
    assert abs(p_learn - p_f32) < 0.5  # bf16 products against the same network in FP32


def test_training_resume_from_checkpoint_is_bitwise(starnt, gpu, sg, oracle_mod):
    """n + n steps with the state saved to the host and reloaded in between give
    the same weights, bit for bit, as 2n steps without a break."""
    fr = sg.Scene("c3_512", width=256, height=256).frame(0)
    from paper_2606_16747_amd import learn
    x, y = learn.pairs_from(starnt.DeviceFrags.from_frame(fr, max_per_pixel=256))
    assert len(x) >= 8192
    x, y = x[:8192], y[:8192]
    Ws, bs = sg.init_mlp((16, 32, 32, 3), seed=5, out_bias=0.05)
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in zip(Ws, bs)]).astype(np.float32)
    n = flat.size
    ws = starnt.workspace(starnt.starnt_workspace_size(starnt.WS_TRAIN, 4096, 32, 32))
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y).cuda()
    loss = torch.zeros(1, device="cuda")

    def run(state, steps, t0):
        p, m, v, g = state
        tr = starnt.Train(16, 32, 32, 3, starnt.BF16, p.data_ptr(), m.data_ptr(), v.data_ptr(), g.data_ptr())
        for t in range(t0, t0 + steps):
            b = t % 2
            starnt.starnt_train_step(tr, xd[b * 4096:(b + 1) * 4096], yd[b * 4096:(b + 1) * 4096], 4096,
                                     starnt.Adam(1e-3, 0.9, 0.999, 1e-8, t + 1), loss, ws)
        sync()

    def fresh():
        return [torch.from_numpy(flat.copy()).cuda(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"),
                torch.zeros(n, device="cuda")]

    a = fresh()
    run(a, 20, 0)
    b = fresh()
    run(b, 10, 0)
    ckpt = [t.cpu().numpy().copy() for t in b[:3]]          # save (params, m, v)
    c = [torch.from_numpy(t).cuda() for t in ckpt] + [torch.zeros(n, device="cuda")]  # load
    run(c, 10, 10)
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1]) and torch.equal(a[2], c[2])


@pytest.mark.parametrize("dims,batch,act", [((16, 32, 32, 3), 1000, 0), ((16, 64, 32, 3), 4097, 0),
                                            ((16, 32, 64, 3), 300, 1), ((16, 64, 64, 3), 65536, 0),
                                            ((16, 16, 32, 3), 777, 0)])
def test_bf16_step_on_matrix_cores(starnt, gpu, sg, oracle_mod, dims, batch, act):
    """The BF16 step (hidden widths 32/64 on the matrix cores; a 16-wide layer
    takes the vector-unit kernel with the same rounding points): its gradient
    points where the FP64 oracle's does (cosine > 0.999, relative L2 < 0.05,
    the bar of bf16 operands), its loss matches within 2%, batches that fill no
    whole block are handled, and a step repeated on the same state is
    bit-identical."""
    fr = sg.Scene("c3_512", width=128, height=128, num_tris=200).frame(0)
    o = oracle_mod.frame_of(fr)
    x = oracle_mod.features(o["lay"], o["tail"])
    keep = o["lay"][:, 0] >= 3
    x, yv = x[keep], o["fstar"][keep]
    rng = np.random.default_rng(batch)
    idx = rng.choice(len(x), batch, replace=len(x) < batch)
    x = x[idx].astype(np.float32)
    y = yv[idx].astype(np.float32)
    # standardised inputs, as the training driver feeds them
    x[:, :5] = (x[:, :5] - x[:, :5].mean(0)) / np.maximum(x[:, :5].std(0), 1e-6)
    if act == 1:
        y = np.clip(y, 0.0, 1.0)
    Ws, bs = sg.init_mlp(dims, seed=7, out_bias=0.1)
    params = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in zip(Ws, bs)]).astype(np.float32)
    n = params.size
    h1, h2 = dims[1], dims[2]
    ws = starnt.workspace(starnt.starnt_workspace_size(starnt.WS_TRAIN, batch, h1, h2))
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    grads, losses = [], []
    for _ in range(2):
        p = torch.from_numpy(params.copy()).cuda()
        m, v, g = (torch.zeros(n, device="cuda") for _ in range(3))
        tr = starnt.Train(16, h1, h2, 3, starnt.BF16, p.data_ptr(), m.data_ptr(), v.data_ptr(), g.data_ptr(), act)
        loss = torch.zeros(1, device="cuda")
        starnt.starnt_train_step(tr, xd, yd, batch, starnt.Adam(1e-3, 0.9, 0.999, 1e-8, 1), loss, ws)
        sync()
        grads.append(to_np(g).copy())
        losses.append(float(to_np(loss)[0]))
    assert np.array_equal(grads[0], grads[1]) and losses[0] == losses[1]
    lw, gw = oracle_mod.loss_grad(dims, params.astype(np.float64), x, y, act=act)
    gg = grads[0].astype(np.float64)
    cos = gg @ gw / (np.linalg.norm(gg) * np.linalg.norm(gw))
    assert cos > 0.999, cos
    assert np.linalg.norm(gg - gw) / np.linalg.norm(gw) < 0.05
    assert abs(losses[0] - lw) <= 0.02 * lw, (losses[0], lw)
