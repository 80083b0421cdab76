"""Pins of two oracle routines that the GPU parity tests lean on:

* the network of Sec. 3.3 evaluated with narrow operands (Mlp.forward_q:
  bf16, and e4m3 with per-layer scales), which every BF16/FP8 parity test
  compares with;
* the mixed-resolution composition of Sec. 3.2 (learned, dfa_learned at
  s < 1): layer 2 and the tail features sampled on their own grids and
  upscaled bilinearly with half-pixel centres.

Every expected value below is written out by hand from the definitions, with
its derivation beside it; none is produced by the routine under test. Each
pin is chosen so that a plausible slip (a bias rounded to the narrow format,
a layer input not re-rounded, scales applied before the bias, (a2, c2)
upscaled instead of (a2, a2 c2), the pass-3 grid sampled at the pass-2
positions, a transposed weight matrix) changes the result.
"""
import numpy as np
import pytest


def _mlp(oracle_mod, Ws, bs):
    return oracle_mod.Mlp([np.asarray(w, np.float32) for w in Ws], [np.asarray(b, np.float32) for b in bs])


# ---------------------------------------------------------------------------
# narrow-operand network (Sec. 3.3 network; bf16 / e4m3 operands, FP64 sums)

def test_bf16_forward_hand_example(oracle_mod):
    """2-2-1-1 network, bf16 operands, biases and sums exact.

    layer 1: x = (1, 3) (bf16-exact), W1 = [[0.5, 0.25], [1, -1]],
      b1 = (0.1f, 4): h1 = (0.5 + 0.75 + 0.1f, 1 - 3 + 4)
                         = (1.350000001490116..., 2)
    layer 2 rounds its input: bf16(1.3500000015) = 1 + 45/128 = 1.3515625
      (0.35 * 128 = 44.8 -> 45); W2 = [[1, 0]], b2 = 0: h2 = 1.3515625
    layer 3: bf16(h2) = h2; W3 = [[2]], b3 = 0.1f (bias NOT rounded):
      y = 2.703125 + 0.100000001490116119384765625
        = 2.803125001490116119384765625 = 376229069 / 2^27
    A bias rounded to bf16 (0.10009765625) gives 2.80322265625; a layer-2
    input left unrounded gives 2.80000000447; W1 transposed gives h1 =
    (3.6, 1.25) and y = 7.3."""
    m = _mlp(oracle_mod, [[[0.5, 0.25], [1.0, -1.0]], [[1.0, 0.0]], [[2.0]]],
             [[0.1, 4.0], [0.0], [0.1]])
    y = m.forward_q(np.array([[1.0, 3.0]]), 1)
    assert y[0, 0] == 376229069 / 2 ** 27
    # the unquantised forward differs exactly by the re-rounding of h1
    assert abs(m.forward(np.array([[1.0, 3.0]]))[0, 0] - 2.8000000044703484) < 1e-15


def test_e4m3_forward_hand_example(oracle_mod):
    """2-1-1-1 network, e4m3 operands with per-layer scales (sa, sw);
    layer l computes (sum q(a / sa) q(W / sw)) sa sw + b, then ReLU.

    layer 1: x = (3, 5), sa1 = 2 -> q(1.5, 2.5) = (1.5, 2.5);
      W1 = [[0.75, 0.5]], sw1 = 0.25 -> q(3, 2) = (3, 2);
      sum = 4.5 + 5 = 9.5; * sa1 sw1 = 0.5 -> 4.75; + b1 0.25 -> 5
      (scales applied after the bias would give 4.875)
    layer 2: q(5 / 3) = q(1.6667): neighbours 1.625 and 1.75 -> 1.625
      (unrounded would carry 1.6667); W2 = [[1.5]], sw2 = 1 -> 1.5;
      sum = 2.4375; * 3 -> 7.3125; + b2 -0.3125 -> 7
    layer 3: q(7 / 1) = 7; W3 = [[0.3f]], sw3 = 0.1:
      q(0.3f / 0.1) = q(3.0000001) = 3; sum = 21; * 0.1 -> 2.1;
      + b3 0.05f -> 2.1500000007450581"""
    m = _mlp(oracle_mod, [[[0.75, 0.5]], [[1.5]], [[0.3]]], [[0.25], [-0.3125], [0.05]])
    sa = np.array([2.0, 3.0, 1.0])
    sw = np.array([0.25, 1.0, 0.1])
    y = m.forward_q(np.array([[3.0, 5.0]]), 2, sa, sw)
    assert abs(y[0, 0] - 2.1500000007450581) < 1e-15
    # the same layer-1 sum with the bias inside the scaled sum lands elsewhere
    assert abs(y[0, 0] - ((9.5 + 0.25) * 0.5)) > 1.0


@pytest.mark.parametrize("qmode", [1, 2])
def test_narrow_forward_equals_fp64_on_exact_operands(oracle_mod, qmode):
    """Special case: when every operand and activation is representable in the
    narrow format (small integers; for e4m3 power-of-two scales that keep
    them on the e4m3 grid), the narrow forward must equal the FP64 forward
    exactly. Weights are random and non-symmetric, so a transposed or
    misindexed operand would differ from the FP64 forward (itself pinned by
    the closed-form and finite-difference tests)."""
    rng = np.random.default_rng(11 + qmode)
    dims = (4, 4, 4, 2)
    Ws = [rng.integers(-1, 2, size=(dims[l + 1], dims[l])).astype(np.float32) for l in range(3)]
    bs = [rng.integers(-1, 2, size=dims[l + 1]).astype(np.float32) for l in range(3)]
    m = _mlp(oracle_mod, Ws, bs)
    x = rng.integers(0, 2, size=(64, 4)).astype(np.float64)
    want = m.forward(x)
    # activations: layer 1 <= 5, layer 2 <= 21 only if all ones; bound them
    # below 16 by construction check (integers <= 16 lie on the e4m3 grid)
    h1 = np.maximum(x @ Ws[0].T.astype(np.float64) + bs[0], 0)
    h2 = np.maximum(h1 @ Ws[1].T.astype(np.float64) + bs[1], 0)
    assert h1.max() <= 16 and h2.max() <= 16
    if qmode == 1:
        got = m.forward_q(x, 1)
    else:
        # q(a / sa) exact for integers <= 16 over sa in {1, 2, 4}; q(W / sw)
        # exact for W in {-1, 0, 1} over sw in {0.5, 1, 2}
        Ws2 = [w * s for w, s in zip(Ws, (0.5, 1.0, 2.0))]
        m = _mlp(oracle_mod, Ws2, bs)
        want = m.forward(x)
        got = m.forward_q(x, 2, np.array([1.0, 2.0, 4.0]), np.array([0.5, 1.0, 2.0]))
    np.testing.assert_array_equal(got, want)


# ---------------------------------------------------------------------------
# mixed resolution (Sec. 3.2): sampling and bilinear upscale of passes 2, 3

def _rows(W, H, n=5):
    lay = np.tile([n, 0.25, 0.4, 0.1, 0.2, 0.3, 0.6, 0.9, 0.5, 0.1], (W * H, 1)).astype(np.float64)
    tail = np.tile([1.1, 0.3, 0.5, 0.2, 0.35, 0.0], (W * H, 1)).astype(np.float64)
    tavg = np.tile([0.4, 0.5, 0.3, 0.55], (W * H, 1)).astype(np.float64)
    return lay, tail, tavg


@pytest.mark.parametrize("grids", [(5, 3, 4, 2), (1, 1, 1, 1), (13, 7, 3, 5), (7, 2, 13, 7)])
def test_identical_lists_give_the_full_resolution_result(oracle_mod, sg, grids):
    """Every pixel holding the same list: each grid holds one value, its
    bilinear upscale is that value (weights sum to 1), so every grid pair must
    give the full-resolution result, for the STAR-NT composite in all modes
    and for the DFAOIT input."""
    W, H = 13, 7
    lay, tail, tavg = _rows(W, H)
    Ws, bs = sg.init_mlp((16, 32, 32, 3), out_bias=0.05)
    mlp = oracle_mod.Mlp(Ws, bs)
    full = (W, H, W, H)
    for mode in (oracle_mod.MODE_LEARNED, oracle_mod.MODE_F0, oracle_mod.MODE_FAVG):
        a = oracle_mod.learned(lay, tail, W, H, grids, mlp if mode == oracle_mod.MODE_LEARNED else None, mode)
        b = oracle_mod.learned(lay, tail, W, H, full, mlp if mode == oracle_mod.MODE_LEARNED else None, mode)
        for u, v in zip(a, b):
            np.testing.assert_allclose(u, v, rtol=0, atol=1e-12)
    da = oracle_mod.dfa_learned(lay, tail, tavg, W, H, grids, None, bg=(0.3, 0.6, 0.9))
    db = oracle_mod.dfa_learned(lay, tail, tavg, W, H, full, None, bg=(0.3, 0.6, 0.9))
    for u, v in zip(da, db):
        np.testing.assert_allclose(u, v, rtol=0, atol=1e-12)


def _six_pixel_frame():
    """A 6 x 1 frame, N = 4 everywhere; layer 1 a1 = 0.5, c1 = 0.2 (grey).
    Layer 2: pixel 1 a2 = 0.5, c2 = red; pixel 4 a2 = 0.75, c2 = green;
    the other pixels a2 = 0.3, c2 = blue (never sampled by a 2-wide grid).
    Tail: A = 1 everywhere so Ctilde = S; pixels 1, 3, 5 (the 3-wide grid's
    samples) t = 0.2, 0.5, 0.8, Ctilde = red, green, blue; pixels 0, 2, 4
    t = 0.9, Ctilde = (0.5, 0.5, 0.5). Tail means: pixels 1, 3, 5 colour
    (0.1, 0, 0), (0, 0.2, 0), (0, 0, 0.3), opacity 0.2, 0.4, 0.6; others 0.9."""
    lay = np.zeros((6, 10))
    lay[:, 0] = 4
    lay[:, 1] = 0.5
    lay[:, 2] = 0.5
    lay[:, 3:6] = 0.2
    lay[:, 6] = 0.3
    lay[:, 7:10] = (0.0, 0.0, 1.0)
    lay[1, 6], lay[1, 7:10] = 0.5, (1.0, 0.0, 0.0)
    lay[4, 6], lay[4, 7:10] = 0.75, (0.0, 1.0, 0.0)
    tail = np.zeros((6, 6))
    tail[:, 0] = 1.0
    tail[:, 1:4] = 0.5
    tail[:, 4] = 0.9
    for p, t, c in ((1, 0.2, (1, 0, 0)), (3, 0.5, (0, 1, 0)), (5, 0.8, (0, 0, 1))):
        tail[p, 1:4] = c
        tail[p, 4] = t
    tavg = np.full((6, 4), 0.9)
    tavg[1] = (0.1, 0.0, 0.0, 0.2)
    tavg[3] = (0.0, 0.2, 0.0, 0.4)
    tavg[5] = (0.0, 0.0, 0.3, 0.6)
    return lay, tail, tavg


# Pass-2 grid of width 2 over W = 6 samples pixels floor((2i+1) 6 / 4) = 1, 4;
# upscale coordinate u = ((2x+1) 2 - 6) / 12 = (x - 1) / 3, so the weights of
# (g0, g1) per pixel are: x=0 (1, 0) [clamped], 1 (1, 0), 2 (2/3, 1/3),
# 3 (1/3, 2/3), 4 (0, 1), 5 (0, 1) [clamped].
W2_WEIGHTS = [(1, 0), (1, 0), (2 / 3, 1 / 3), (1 / 3, 2 / 3), (0, 1), (0, 1)]
# Pass-3 grid of width 3 samples pixels floor((2i+1) 6 / 6) = 1, 3, 5;
# u = ((2x+1) 3 - 6) / 12 = (2x - 1) / 4: weights of (g0, g1, g2):
W3_WEIGHTS = [(1, 0, 0), (3 / 4, 1 / 4, 0), (1 / 4, 3 / 4, 0), (0, 3 / 4, 1 / 4), (0, 1 / 4, 3 / 4), (0, 0, 1)]


def test_pass2_upscale_blends_premultiplied_layer(oracle_mod):
    """f = 0, background 0: C = a1 c1 + (1 - a1) up(a2 c2). Hand values:
    g0 = (a2, a2 c2) = (0.5, 0.5, 0, 0), g1 = (0.75, 0, 0.75, 0);
      x=2: up(a2 c2) = 2/3 (0.5, 0, 0) + 1/3 (0, 0.75, 0) = (1/3, 1/4, 0)
           C = 0.1 + 0.5 (1/3, 1/4, 0) = (4/15, 0.225, 0.1)
      x=3: up(a2 c2) = (1/6, 1/2, 0); C = (1/6 + 1/10 ..) = (0.18333.., 0.35, 0.1)
    Upscaling (a2, c2) and multiplying would give at x = 3: a2 = 2/3,
    c2 = (1/3, 2/3, 0), a2 c2 = (2/9, 4/9, 0), C = (0.2111, 0.3222, 0.1)."""
    lay, tail, _ = _six_pixel_frame()
    rgb, _, _ = oracle_mod.learned(lay, tail, 6, 1, (2, 1, 6, 1), None, oracle_mod.MODE_F0, bg=(0.0, 0.0, 0.0))
    want = np.array([
        [0.1 + 0.25, 0.1, 0.1],                # x=0: g0 only: 0.1 + 0.5 (0.5, 0, 0)
        [0.1 + 0.25, 0.1, 0.1],                # x=1: g0
        [0.1 + 1 / 6, 0.1 + 0.125, 0.1],       # x=2
        [0.1 + 1 / 12, 0.1 + 0.25, 0.1],       # x=3
        [0.1, 0.1 + 0.375, 0.1],               # x=4: g1 only: 0.1 + 0.5 (0, 0.75, 0)
        [0.1, 0.1 + 0.375, 0.1],               # x=5: g1
    ])
    np.testing.assert_allclose(rgb, want, rtol=0, atol=1e-15)
    # with a background, T2 t_tail C_b enters with the upscaled a2 and the
    # pass-3 t_tail: x=3: a2 = 1/3 0.5 + 2/3 0.75 = 2/3, T2 = 0.5 / 3 = 1/6,
    # t_tail = 3/4 0.5 + 1/4 0.8 = 0.575 -> background term 0.575 / 6
    rgb1, _, _ = oracle_mod.learned(lay, tail, 6, 1, (2, 1, 3, 1), None, oracle_mod.MODE_F0, bg=(1.0, 1.0, 1.0))
    np.testing.assert_allclose(rgb1[3], want[3] + 0.575 / 6, rtol=0, atol=1e-15)


def test_pass3_upscale_uses_its_own_grid(oracle_mod):
    """The network input x = (N, t_tail, Ctilde) is sampled on the pass-3 grid
    (pixels 1, 3, 5 for width 3) and upscaled with that grid's weights, even
    when the pass-2 grid differs (width 2, pixels 1 and 4). Hand values:
      x=2: 1/4 g0 + 3/4 g1 -> t = 0.05 + 0.375 = 0.425, Ctilde = (1/4, 3/4, 0)
      x=4: 1/4 g1 + 3/4 g2 -> t = 0.125 + 0.6 = 0.725, Ctilde = (0, 1/4, 3/4)
    and f_avg = Ctilde (1 - t) enters eq (3) with T2 = (1 - a1)(1 - up(a2))."""
    lay, tail, _ = _six_pixel_frame()
    rgb, xf, f = oracle_mod.learned(lay, tail, 6, 1, (2, 1, 3, 1), None, oracle_mod.MODE_FAVG,
                                    bg=(0.0, 0.0, 0.0))
    want_t = [0.2, 0.2 * 0.75 + 0.5 * 0.25, 0.425, 0.5 * 0.75 + 0.8 * 0.25, 0.725, 0.8]
    want_c = [(1, 0, 0), (0.75, 0.25, 0), (0.25, 0.75, 0), (0, 0.75, 0.25), (0, 0.25, 0.75), (0, 0, 1)]
    np.testing.assert_allclose(xf[:, 0], 4.0, rtol=0, atol=0)
    np.testing.assert_allclose(xf[:, 1], want_t, rtol=0, atol=1e-15)
    np.testing.assert_allclose(xf[:, 2:5], want_c, rtol=0, atol=1e-15)
    assert not xf[:, 5:].any()
    np.testing.assert_allclose(f, np.array(want_c) * (1 - np.array(want_t))[:, None], rtol=0, atol=1e-15)
    # x=2: a2 = 2/3 0.5 + 1/3 0.75 = 7/12, T2 = 0.5 * 5/12 = 5/24;
    # C = 0.1 + 0.5 (1/3, 1/4, 0) + 5/24 f
    f2 = np.array([0.25, 0.75, 0.0]) * 0.575
    np.testing.assert_allclose(rgb[2], 0.1 + 0.5 * np.array([1 / 3, 1 / 4, 0]) + 5 / 24 * f2, rtol=0, atol=1e-15)


def test_gating_by_full_resolution_count(oracle_mod):
    """The full-resolution N gates the upscaled terms: a pixel with N = 2 gets
    no tail (f = 0, t_tail = 1) and one with N = 1 no second layer, whatever
    its neighbours' grid samples hold."""
    lay, tail, _ = _six_pixel_frame()
    lay[2, 0] = 2
    lay[3, 0] = 1
    rgb, xf, f = oracle_mod.learned(lay, tail, 6, 1, (2, 1, 3, 1), None, oracle_mod.MODE_FAVG,
                                    bg=(1.0, 1.0, 1.0))
    assert not f[2].any() and not f[3].any()
    # x=2: C = 0.1 + 0.5 (1/3, 1/4, 0) + T2 * 1 * 1, T2 = 0.5 (1 - 7/12)
    np.testing.assert_allclose(rgb[2], 0.1 + 0.5 * np.array([1 / 3, 1 / 4, 0]) + 0.5 * 5 / 12, rtol=0, atol=1e-15)
    # x=3: no layer 2: C = 0.1 + 0.5 * 1 * 1
    np.testing.assert_allclose(rgb[3], [0.6, 0.6, 0.6], rtol=0, atol=1e-15)


def test_dfa_input_upscale_hand_values(oracle_mod):
    """DFAOIT input (Sec. 3.3) on the same frame, pass 2 width 2, pass 3
    width 3: x = (a1 c1 + (1 - a1) up(a2 c2), up(mean c), up(mean a),
    up(S), up(N)). Hand values at x = 3 (pass-2 weights 1/3, 2/3; pass-3
    weights 0, 3/4, 1/4 of samples 1, 3, 5):
      exact2 = 0.1 + 0.5 (1/6, 1/2, 0) = (0.18333.., 0.35, 0.1)
      mean colour = 3/4 (0, 0.2, 0) + 1/4 (0, 0, 0.3) = (0, 0.15, 0.075)
      mean opacity = 3/4 0.4 + 1/4 0.6 = 0.45
      S = 3/4 green + 1/4 blue = (0, 0.75, 0.25); N = 4."""
    lay, tail, tavg = _six_pixel_frame()
    _, x, _ = oracle_mod.dfa_learned(lay, tail, tavg, 6, 1, (2, 1, 3, 1), None, bg=(0.0, 0.0, 0.0))
    want3 = [0.1 + 1 / 12, 0.35, 0.1, 0.0, 0.15, 0.075, 0.45, 0.0, 0.75, 0.25, 4.0]
    np.testing.assert_allclose(x[3, :11], want3, rtol=0, atol=1e-15)
    assert not x[:, 11:].any()
    # x = 0: clamped to the first samples of both grids
    want0 = [0.35, 0.1, 0.1, 0.1, 0.0, 0.0, 0.2, 1.0, 0.0, 0.0, 4.0]
    np.testing.assert_allclose(x[0, :11], want0, rtol=0, atol=1e-15)
