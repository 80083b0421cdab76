"""Pins of the oracle's DFAOIT variant (Sec. 3.3, eq (2)): the tail means,
the ten-feature input, the sigmoid-output network and its gradient, and the
composite that adds the background through all fragments."""
import numpy as np
import pytest

from csr_util import make_csr, random_lists


def test_tail_means_worked_example(oracle_mod):
    """Red, green, blue, white at depths 0.1..0.4 (stored shuffled): the tail
    is blue and white, so the mean colour is (1/2, 1/2, 1) and the mean
    opacity the mean of their alphas."""
    frs = [(0.3, 3, 0.0, 0.0, 1.0, 0.25), (0.1, 1, 1.0, 0.0, 0.0, 0.5),
           (0.4, 4, 1.0, 1.0, 1.0, 0.75), (0.2, 2, 0.0, 1.0, 0.0, 0.5)]
    o = oracle_mod.frame(*make_csr([frs], 1, 1), 1, 1, want=("tavg", "lay", "tail"))
    np.testing.assert_allclose(o["tavg"][0], [0.5, 0.5, 1.0, 0.5], rtol=0, atol=1e-15)
    x = oracle_mod.dfa_features(o["lay"], o["tail"], o["tavg"])[0]
    # exact two-layer colour: red at 1/2 over green at 1/2 -> (1/2, 1/4, 0)
    np.testing.assert_allclose(x[0:3], [0.5, 0.25, 0.0], atol=1e-15)
    np.testing.assert_allclose(x[3:7], [0.5, 0.5, 1.0, 0.5], atol=1e-15)
    # accumulated premultiplied tail colour: 0.25 blue + 0.75 white
    np.testing.assert_allclose(x[7:10], [0.75, 0.75, 1.0], atol=1e-15)
    assert x[10] == 4 and np.all(x[11:] == 0)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 9])
def test_tail_means_uniform_lists(oracle_mod, n):
    c, a = (0.2, 0.4, 0.6), 0.3
    lists = [[(0.1 * (k + 1), k, *c, a) for k in range(n)]]
    o = oracle_mod.frame(*make_csr(lists, 1, 1), 1, 1, want=("tavg",))
    want = [*c, a] if n >= 3 else [0.0, 0.0, 0.0, 0.0]
    np.testing.assert_allclose(o["tavg"][0], np.float32(want).astype(np.float64) if n >= 3 else want, atol=1e-7)


def test_tail_means_are_order_free(oracle_mod):
    rng = np.random.default_rng(8)
    lists = random_lists(rng, 8, 8, 12)
    a = oracle_mod.frame(*make_csr(lists, 8, 8), 8, 8, want=("tavg",))["tavg"]
    b = oracle_mod.frame(*make_csr([l[::-1] for l in lists], 8, 8), 8, 8, want=("tavg",))["tavg"]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("b3,want_relu,want_sig", [(0.0, 0.0, 0.5), (np.log(3.0), np.log(3.0), 0.75),
                                                   (-2.0, 0.0, 1.0 / (1.0 + np.exp(2.0)))])
def test_output_activation_bias_only(oracle_mod, b3, want_relu, want_sig):
    """With zero weights the output is act(b3): ReLU or the logistic sigmoid."""
    Ws = [np.zeros((8, 16), np.float32), np.zeros((8, 8), np.float32), np.zeros((3, 8), np.float32)]
    bs = [np.ones(8, np.float32), np.ones(8, np.float32), np.full(3, b3, np.float32)]
    x = np.random.default_rng(0).random((4, 16))
    b3f = float(np.float32(b3))
    np.testing.assert_allclose(oracle_mod.Mlp(Ws, bs, act=0).forward(x), max(b3f, 0.0), atol=1e-15)
    np.testing.assert_allclose(oracle_mod.Mlp(Ws, bs, act=1).forward(x), 1.0 / (1.0 + np.exp(-b3f)), atol=1e-15)
    assert abs(1.0 / (1.0 + np.exp(-b3f)) - want_sig) < 1e-7 and abs(max(b3f, 0.0) - want_relu) < 1e-7


def test_sigmoid_gradient_matches_finite_differences(oracle_mod, sg):
    dims = (16, 8, 8, 3)
    Ws, bs = sg.init_mlp(dims, seed=9, out_bias=0.1)
    w = np.concatenate([np.concatenate([a.ravel(), b.ravel()]) for a, b in zip(Ws, bs)]).astype(np.float64)
    rng = np.random.default_rng(2)
    x = rng.random((32, 16))
    y = rng.random((32, 3))
    loss, g = oracle_mod.loss_grad(dims, w, x, y, act=1)
    for i in rng.choice(w.size, 40, replace=False):
        e = np.zeros_like(w)
        e[i] = 1e-6
        fd = (oracle_mod.loss_grad(dims, w + e, x, y, act=1)[0] - oracle_mod.loss_grad(dims, w - e, x, y, act=1)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])
    # the forward of the loss is the sigmoid network's
    f = oracle_mod.Mlp(Ws, bs, act=1).forward(x)
    assert abs(loss - np.mean((f - y) ** 2)) < 1e-12


def test_dfa_composite_with_the_exact_colour_is_exact(oracle_mod):
    """With C_t equal to the exact colour over a black background, eq (2)
    reproduces the exact composite over any background."""
    rng = np.random.default_rng(3)
    lists = random_lists(rng, 9, 9, 14)
    csr = make_csr(lists, 9, 9)
    bg = (0.3, 0.9, 0.1)
    o = oracle_mod.frame(*csr, 9, 9, bg=bg, want=("rgb", "lay", "tail"))
    Ct = oracle_mod.frame(*csr, 9, 9, bg=(0.0, 0.0, 0.0), want=("rgb",))["rgb"]
    out = oracle_mod.dfa_composite(o["lay"], o["tail"], Ct, bg)
    np.testing.assert_allclose(out, o["rgb"], rtol=0, atol=1e-13)


def test_dfa_mixed_resolution_reduces_to_full_resolution(oracle_mod, sg):
    """At s = 1 the upscale is the identity: the mixed-resolution DFAOIT path
    equals dfa_features and dfa_composite at full resolution."""
    fr = sg.Scene("c1_256", width=48, height=40, num_tris=30).frame(0)
    o = oracle_mod.frame_of(fr, want=("rgb", "lay", "tail", "tavg"))
    Ws, bs = sg.init_mlp((16, 8, 8, 3), seed=4, out_bias=0.1)
    m = oracle_mod.Mlp(Ws, bs, act=1)
    W, H = fr.width, fr.height
    rgb, x, f = oracle_mod.dfa_learned(o["lay"], o["tail"], o["tavg"], W, H, (W, H, W, H), m, bg=(0.5, 0.5, 0.5))
    x0 = oracle_mod.dfa_features(o["lay"], o["tail"], o["tavg"])
    t = o["lay"][:, 0] >= 3
    np.testing.assert_allclose(x[t], x0[t], rtol=0, atol=1e-12)
    assert np.all(x[~t] == 0)
    f0 = m.forward(x0)
    want = oracle_mod.dfa_composite(o["lay"], o["tail"], f0, (0.5, 0.5, 0.5))
    np.testing.assert_allclose(rgb, want, rtol=0, atol=1e-12)
