"""Oracle pins for the per-sample weighted training loss and for the
rounding-ambiguity flags of the narrow-operand network forward.

Weighted loss (the composite-space reading of the MSE of Sec. 3.3: eq (3)
scales the network output by T2, so weighting each sample's squared error by
T2^2 makes the loss the mean squared error of the composite's tail term):
closed forms on zero-weight networks, equality with the plain loss for unit
weights and with a single sample's loss for a one-hot weight, and central
finite differences of a randomly weighted loss.

Ambiguity flags: values placed by hand at and away from bf16 and e4m3
rounding boundaries."""
import numpy as np
import pytest

from test_oracle_qt_reproj_train import _kink_free_batch


def _zero_net(b3):
    dims = (16, 4, 4, 3)
    n = 4 * 16 + 4 + 16 + 4 + 12 + 3
    w = np.zeros(n)
    w[-3:] = b3
    return dims, w


def test_weighted_loss_closed_form(oracle_mod):
    """Zero weights: f = relu(b3); loss = sum_k wt_k sum_o (f_o - y_ko)^2 / (3 B)
    and d/db3_o = 2 sum_k wt_k (f_o - y_ko) / (3 B) on live outputs."""
    dims, w = _zero_net((0.5, -1.0, 0.25))
    rng = np.random.default_rng(0)
    x = rng.random((5, 16))
    y = rng.random((5, 3))
    wt = np.array([0.0, 1.0, 0.25, 2.0, 0.5])
    loss, g = oracle_mod.loss_grad(dims, w, x, y, wt=wt)
    f = np.array([0.5, 0.0, 0.25])
    want = (wt[:, None] * (f - y) ** 2).sum() / 15.0
    assert abs(loss - want) < 1e-15
    np.testing.assert_allclose(g[-3:], [2 * (wt * (0.5 - y[:, 0])).sum() / 15, 0.0,
                                        2 * (wt * (0.25 - y[:, 2])).sum() / 15], atol=1e-15)
    assert np.all(g[:-3] == 0)


def test_unit_weights_give_the_plain_loss(oracle_mod, sg):
    dims = (16, 8, 8, 3)
    rng = np.random.default_rng(1)
    Ws, bs = sg.init_mlp(dims, seed=77, out_bias=0.2)
    w = np.concatenate([np.concatenate([a.ravel(), b.ravel()]) for a, b in zip(Ws, bs)]).astype(np.float64)
    x = rng.random((9, 16))
    y = rng.random((9, 3))
    l0, g0 = oracle_mod.loss_grad(dims, w, x, y)
    l1, g1 = oracle_mod.loss_grad(dims, w, x, y, wt=np.ones(9))
    assert l0 == l1 and np.array_equal(g0, g1)


def test_one_hot_weight_is_one_sample_scaled(oracle_mod, sg):
    """wt = B e_k: exactly the plain loss and gradient of sample k alone."""
    dims = (16, 8, 8, 3)
    rng = np.random.default_rng(2)
    Ws, bs = sg.init_mlp(dims, seed=78, out_bias=0.2)
    w = np.concatenate([np.concatenate([a.ravel(), b.ravel()]) for a, b in zip(Ws, bs)]).astype(np.float64)
    x = rng.random((8, 16))
    y = rng.random((8, 3))
    wt = np.zeros(8)
    wt[3] = 8.0
    l1, g1 = oracle_mod.loss_grad(dims, w, x, y, wt=wt)
    l0, g0 = oracle_mod.loss_grad(dims, w, x[3:4], y[3:4])
    assert abs(l1 - l0) <= 1e-15 * max(1.0, l0)
    np.testing.assert_allclose(g1, g0, rtol=1e-13, atol=1e-16)


def test_weighted_gradient_central_differences(oracle_mod):
    dims = (16, 12, 10, 3)
    rng = np.random.default_rng(3)
    n = 12 * 16 + 12 + 10 * 12 + 10 + 3 * 10 + 3
    w = rng.normal(scale=0.4, size=n)
    w[-3:] = 0.5
    x = _kink_free_batch(dims, w, rng, 6)
    y = rng.random((6, 3))
    wt = rng.random(6) ** 2
    loss, g = oracle_mod.loss_grad(dims, w, x, y, wt=wt)
    h = 1e-6
    for i in rng.choice(n, 60, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (oracle_mod.loss_grad(dims, wp, x, y, wt=wt)[0] - oracle_mod.loss_grad(dims, wm, x, y, wt=wt)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def _one_input_net(sg, w1=1.0):
    """16-1-1-1... widths of at least 1: unit weights pass input 0 through."""
    dims = (16, 1, 1, 3)
    Ws = [np.zeros((1, 16), np.float32), np.ones((1, 1), np.float32), np.ones((3, 1), np.float32)]
    Ws[0][0, 0] = w1
    bs = [np.zeros(1, np.float32), np.zeros(1, np.float32), np.zeros(3, np.float32)]
    return Ws, bs


def test_ambiguity_flags_bf16_inputs(oracle_mod, sg):
    """bf16 near 1.5: representable neighbours 1.5 and 1.5078125, midpoint
    1.50390625. An input at the midpoint is flagged (bit 0), one at a
    representable value or half a step from the midpoint is not."""
    Ws, bs = _one_input_net(sg)
    om = oracle_mod.Mlp(Ws, bs)
    x = np.zeros((3, 16))
    x[:, 0] = (1.50390625, 1.5, 1.50390625 + 0.001953125)
    _, amb = om.forward_q_amb(x, 1, tol_in=1e-6, tol_h=0.0)
    assert list(amb) == [1, 0, 0]
    # with no move allowed nothing is flagged
    _, amb = om.forward_q_amb(x, 1, tol_in=0.0, tol_h=0.0)
    assert list(amb) == [0, 0, 0]


def test_ambiguity_flags_hidden_activation(oracle_mod, sg):
    """Input 1, first-layer weight 0.5 (bf16 values) and bias b: the first
    activation is 0.5 + b exactly. bf16 neighbours 0.5 and 0.50390625 have the
    midpoint 0.501953125: with b = 0.001953125 the activation sits on it and is
    flagged (bit 1); with b = 0.00390625 it is a bf16 value and is not."""
    x = np.zeros((1, 16))
    x[0, 0] = 1.0
    flags = []
    for b in (0.001953125, 0.00390625):
        Ws, bs = _one_input_net(sg, w1=0.5)
        bs[0][0] = b
        _, amb = oracle_mod.Mlp(Ws, bs).forward_q_amb(x, 1, tol_in=0.0, tol_h=1e-6)
        flags.append(int(amb[0]))
    assert flags == [2, 0]


def test_ambiguity_flags_e4m3(oracle_mod, sg):
    """e4m3 near 1: neighbours 1 and 1.125, midpoint 1.0625; with input
    scale 2 the input 2.125 maps to the midpoint and is flagged, 2.25 (an
    e4m3 value after scaling) is not. A zero activation (ReLU kink) is never
    flagged: its two roundings differ by no more than the move."""
    Ws, bs = _one_input_net(sg)
    om = oracle_mod.Mlp(Ws, bs)
    x = np.zeros((3, 16))
    x[:, 0] = (2.125, 2.25, 0.0)
    sa = np.array([2.0, 1.0, 1.0])
    sw = np.array([1.0, 1.0, 1.0])
    _, amb = om.forward_q_amb(x, 2, sa, sw, tol_in=1e-6, tol_h=1e-6)
    assert list(amb) == [1, 0, 0]
