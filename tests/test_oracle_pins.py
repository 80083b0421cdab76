"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form,
an exact rational brute force on tiny inputs, an invariant, or a property the
paper states. Equation numbers refer to the STAR-NT paper (arXiv 2606.16747).
"""
from fractions import Fraction

import numpy as np
import pytest

from csr_util import make_csr, random_lists


# ---------------------------------------------------------------------------
# eq (1), eq (3), tail statistics: closed forms

@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 17, 64])
@pytest.mark.parametrize("a", [0.2, 0.5, 0.8])
def test_equal_alpha_layers_closed_form(oracle_mod, n, a):
    """n layers of equal alpha a and colour c: T_N = (1-a)^n,
    C = c (1 - (1-a)^n) + (1-a)^n C_b, t_tail = (1-a)^(n-2), A = (n-2) a,
    Ctilde = c, f* = f_avg = c (1 - (1-a)^(n-2))."""
    c = np.array([0.3, 0.6, 0.9])
    bg = np.array([1.0, 0.5, 0.0])
    rng = np.random.default_rng(n)
    zs = rng.permutation(n).astype(np.float32) / max(n, 1)
    lists = [[(float(zs[k]), k, *c, a) for k in range(n)]]
    # a float32 a: use the stored value in the closed form
    a32 = float(np.float32(a))
    c32 = c.astype(np.float32).astype(np.float64)
    o = oracle_mod.frame(*make_csr(lists, 1, 1), 1, 1, bg=bg)
    TN = (1 - a32) ** n
    np.testing.assert_allclose(o["rgb"][0], c32 * (1 - TN) + TN * bg, rtol=0, atol=1e-12)
    m = max(n - 2, 0)
    tt = (1 - a32) ** m
    np.testing.assert_allclose(o["tail"][0, 4], tt, atol=1e-12)
    np.testing.assert_allclose(o["tail"][0, 0], m * a32, atol=1e-12)
    x = oracle_mod.features(o["lay"], o["tail"])
    if m > 0:
        np.testing.assert_allclose(x[0, 2:5], c32, atol=1e-12)
    else:
        np.testing.assert_array_equal(x[0, 2:5], 0.0)
        assert x[0, 1] == 1.0
    np.testing.assert_allclose(o["fstar"][0], c32 * (1 - tt), atol=1e-12)
    assert x[0, 0] == n


def test_small_lists_have_empty_tail(oracle_mod):
    """Pixels with two or fewer fragments: A = 0, Ctilde = 0, t_tail = 1, f* = 0."""
    rng = np.random.default_rng(7)
    lists = random_lists(rng, 8, 8, 2)
    o = oracle_mod.frame(*make_csr(lists, 8, 8), 8, 8)
    assert np.all(o["tail"][:, 0] == 0)
    assert np.all(o["tail"][:, 4] == 1.0)
    assert np.all(o["fstar"] == 0)
    x = oracle_mod.features(o["lay"], o["tail"])
    assert np.all(x[:, 2:5] == 0)


def _rational_pixel(l, bg):
    """Exact rational front-to-back composite with ranks from pairwise key
    comparisons (no sort): rank_i = #{j : key_j < key_i}."""
    keys = [(Fraction(float(np.float32(z))), pr) for (z, pr, *_r) in l]
    n = len(l)
    rank = [sum(1 for j in range(n) if keys[j] < keys[i]) for i in range(n)]
    order = [None] * n
    for i in range(n):
        order[rank[i]] = i
    vals = [tuple(Fraction(float(np.float32(v))) for v in (r, g, b, a)) for (_z, _p, r, g, b, a) in l]
    T = Fraction(1)
    C = [Fraction(0)] * 3
    Tt = Fraction(1)
    Ft = [Fraction(0)] * 3
    A = Fraction(0)
    S = [Fraction(0)] * 3
    for pos, i in enumerate(order):
        r, g, b, a = vals[i]
        for k, v in enumerate((r, g, b)):
            C[k] += T * a * v
        T *= (1 - a)
        if pos >= 2:
            for k, v in enumerate((r, g, b)):
                Ft[k] += Tt * a * v
                S[k] += a * v
            Tt *= (1 - a)
            A += a
    bgf = [Fraction(float(v)) for v in bg]
    rgb = [C[k] + T * bgf[k] for k in range(3)]
    return rgb, Ft, A, S, Tt, order


@pytest.mark.parametrize("ties", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_8x8(oracle_mod, seed, ties):
    """8x8 frames: exact rational arithmetic with ranks by counting (O(n^2)),
    including frames where equal depths are common (tie-break on primitive id)."""
    rng = np.random.default_rng(seed)
    lists = random_lists(rng, 8, 8, 9, ties=ties)
    csr = make_csr(lists, 8, 8)
    bg = (0.25, 0.5, 1.0)
    o = oracle_mod.frame(*csr, 8, 8, bg=bg)
    offsets = csr[0]
    for p, l in enumerate(lists):
        rgb, Ft, A, S, Tt, order = _rational_pixel(l, bg)
        np.testing.assert_allclose(o["rgb"][p], [float(v) for v in rgb], rtol=0, atol=1e-13)
        np.testing.assert_allclose(o["fstar"][p], [float(v) for v in Ft], rtol=0, atol=1e-13)
        np.testing.assert_allclose(o["tail"][p, 0], float(A), atol=1e-13)
        np.testing.assert_allclose(o["tail"][p, 1:4], [float(v) for v in S], atol=1e-13)
        np.testing.assert_allclose(o["tail"][p, 4], float(Tt), atol=1e-13)
        for k in range(2):
            want = offsets[p] + order[k] if k < len(l) else 0xFFFFFFFF
            assert o["sel"][p, k] == want


def test_decomposition_identity(oracle_mod, sg):
    """eq (3) with the exact tail colour: C = C_exact,2 + T2 f* + T_N C_b holds
    exactly for every pixel (T_N = T2 t_tail)."""
    fr = sg.Scene("c1_256").frame(0)
    bg = np.array([0.9, 0.2, 0.4])
    o = oracle_mod.frame_of(fr, bg=bg)
    L = o["lay"]
    a1, c1, a2, c2 = L[:, 2:3], L[:, 3:6], L[:, 6:7], L[:, 7:10]
    T2 = (1 - a1) * (1 - a2)
    TN = T2 * o["tail"][:, 4:5]
    rec = a1 * c1 + (1 - a1) * a2 * c2 + T2 * o["fstar"] + TN * bg
    np.testing.assert_allclose(rec, o["rgb"], rtol=0, atol=1e-12)


def test_uniform_colour_tail_makes_favg_exact(oracle_mod, sg):
    """If every tail fragment has the same colour c, f* = c (1 - t_tail) = f_avg."""
    fr = sg.Scene("c1_256").frame(0)
    rgba = fr.rgba.copy()
    rgba[:, 0:3] = (0.1, 0.7, 0.4)
    o = oracle_mod.frame(fr.offsets, fr.depth, rgba, fr.prim, fr.width, fr.height)
    x = oracle_mod.features(o["lay"], o["tail"])
    favg = x[:, 2:5] * (1 - x[:, 1:2])
    np.testing.assert_allclose(favg, o["fstar"], atol=1e-12)
    # and the learned composite with f = f_avg reproduces the exact image
    rgb, _, _ = oracle_mod.learned(o["lay"], o["tail"], fr.width, fr.height,
                                   (fr.width, fr.height, fr.width, fr.height), None, oracle_mod.MODE_FAVG)
    np.testing.assert_allclose(rgb, o["rgb"], atol=1e-12)


def test_two_or_fewer_layers_learned_equals_exact(oracle_mod, sg):
    """With N <= 2 the learned composite is exact whatever the network says."""
    fr = sg.Scene("c1_256").frame(0)
    o = oracle_mod.frame_of(fr)
    import scenegen
    Ws, bs = scenegen.init_mlp((16, 32, 32, 3), out_bias=0.3)
    mlp = oracle_mod.Mlp(Ws, bs)
    rgb, _, _ = oracle_mod.learned(o["lay"], o["tail"], fr.width, fr.height,
                                   (fr.width, fr.height, fr.width, fr.height), mlp)
    small = o["lay"][:, 0] <= 2
    assert small.sum() > 1000
    np.testing.assert_allclose(rgb[small], o["rgb"][small], atol=1e-12)


def test_permutation_invariance(oracle_mod, sg):
    """Permuting each pixel's list changes nothing (bit-identical in FP64)."""
    fr = sg.Scene("c1_256").frame(0)
    fr2 = scenegen_shuffled(sg, fr, 11)
    a = oracle_mod.frame_of(fr)
    b = oracle_mod.frame_of(fr2)
    for k in ("rgb", "fstar", "lay", "tail"):
        np.testing.assert_array_equal(a[k], b[k])
    # selected fragments are the same fragments (same depth and primitive)
    for k in range(2):
        ia, ib = a["sel"][:, k], b["sel"][:, k]
        ok = ia != 0xFFFFFFFF
        assert np.all((ib != 0xFFFFFFFF) == ok)
        assert np.array_equal(fr.prim[ia[ok]], fr2.prim[ib[ok]])


def scenegen_shuffled(sg, fr, seed):
    return sg.shuffled(fr, seed)


# ---------------------------------------------------------------------------
# network

def test_mlp_zero_weights_gives_relu_bias(oracle_mod):
    Ws = [np.zeros((32, 16)), np.zeros((32, 32)), np.zeros((3, 32))]
    bs = [np.ones(32), np.ones(32), np.array([0.5, -0.25, 2.0])]
    m = oracle_mod.Mlp(Ws, bs)
    y = m.forward(np.random.default_rng(0).random((10, 16)))
    np.testing.assert_array_equal(y, np.tile([0.5, 0.0, 2.0], (10, 1)))


def test_mlp_identity_path(oracle_mod):
    """Selector weights pass x[0..2] through three ReLU layers unchanged when
    positive and give 0 when negative."""
    W1 = np.zeros((8, 16)); W1[0, 0] = W1[1, 1] = W1[2, 2] = 1
    W2 = np.zeros((8, 8)); W2[0, 0] = W2[1, 1] = W2[2, 2] = 1
    W3 = np.zeros((3, 8)); W3[0, 0] = W3[1, 1] = W3[2, 2] = 1
    m = oracle_mod.Mlp([W1, W2, W3], [np.zeros(8), np.zeros(8), np.zeros(3)])
    x = np.zeros((3, 16))
    x[0, :3] = (0.25, 2.0, 7.5)
    x[1, :3] = (-1.0, 0.5, -0.125)
    y = m.forward(x)
    np.testing.assert_array_equal(y[0], [0.25, 2.0, 7.5])
    np.testing.assert_array_equal(y[1], [0.0, 0.5, 0.0])
    np.testing.assert_array_equal(y[2], [0.0, 0.0, 0.0])


def test_mlp_positive_homogeneity(oracle_mod, sg):
    """With zero biases a ReLU network is positively homogeneous: f(l x) = l f(x)."""
    Ws, _ = sg.init_mlp((16, 32, 32, 3))
    m = oracle_mod.Mlp(Ws, [np.zeros(32), np.zeros(32), np.zeros(3)])
    x = np.random.default_rng(1).normal(size=(50, 16))
    for lam in (0.5, 2.0, 8.0):
        np.testing.assert_allclose(m.forward(lam * x), lam * m.forward(x), rtol=1e-12, atol=1e-14)


def test_mlp_dims_independent_of_zero_inputs(oracle_mod, sg):
    """Zero-padded input columns change nothing: 5 live features + 11 zeros give
    the same output whatever weights multiply the padding."""
    Ws, bs = sg.init_mlp((16, 32, 16, 3), out_bias=0.1)
    x = np.zeros((20, 16))
    x[:, :5] = np.random.default_rng(2).random((20, 5))
    W1b = Ws[0].copy()
    W1b[:, 5:] = 123.0
    a = oracle_mod.Mlp(Ws, bs).forward(x)
    b = oracle_mod.Mlp([W1b, Ws[1], Ws[2]], bs).forward(x)
    np.testing.assert_array_equal(a, b)


def test_bf16_rounding_definition(oracle_mod):
    """bfloat16: 8 exponent bits, 7 stored mantissa bits, ties to even."""
    r = oracle_mod.round_bf16
    assert r(1.0) == 1.0
    assert r(1.0 + 2.0 ** -8) == 1.0                  # tie -> even (1.0)
    assert r(1.0 + 3 * 2.0 ** -8) == 1.0 + 2 * 2.0 ** -7  # tie -> even (mantissa 2)
    assert r(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert r(-2.5) == -2.5
    # every bf16 value is a fixed point; midpoints go to the even neighbour
    for bits in range(0x3F80, 0x4000):
        v = float(np.array([bits << 16], np.uint32).view(np.float32)[0])
        assert r(v) == v
        nxt = float(np.array([(bits + 1) << 16], np.uint32).view(np.float32)[0])
        mid = (v + nxt) / 2
        want = v if (bits % 2 == 0) else nxt
        assert r(mid) == want


def _e4m3_values():
    """All finite OCP E4M3 values decoded from their bit patterns."""
    vals = []
    for b in range(256):
        s = -1.0 if b & 0x80 else 1.0
        e = (b >> 3) & 0xF
        m = b & 0x7
        if e == 15 and m == 7:
            continue  # NaN
        v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
        vals.append(s * v)
    return sorted(set(vals))


def test_e4m3_rounding_definition(oracle_mod):
    """OCP E4M3 (max 448, subnormal step 2^-9): every code decodes to a fixed
    point of the rounding; midpoints round to the neighbour with an even
    mantissa; out-of-range values saturate to +-448."""
    r = oracle_mod.round_e4m3
    vals = _e4m3_values()
    assert max(vals) == 448.0 and min(v for v in vals if v > 0) == 2.0 ** -9
    pos = [v for v in vals if v >= 0]
    assert len(pos) == 127
    for v in vals:
        assert r(v) == v
    for a, b in zip(pos[:-1], pos[1:]):
        mid = (a + b) / 2
        # the even neighbour: mantissa field even
        def mant(v):
            if v < 2.0 ** -6:
                return int(round(v / 2.0 ** -9))
            e = int(np.floor(np.log2(v)))
            return int(round((v / 2.0 ** e - 1) * 8))
        want = a if mant(a) % 2 == 0 else b
        assert r(mid) == want, (a, b)
        assert r(a + (b - a) * 0.3) == a
        assert r(a + (b - a) * 0.7) == b
    assert r(1000.0) == 448.0 and r(-1e9) == -448.0


# ---------------------------------------------------------------------------
# mixed resolution

def test_grid_and_sampling(oracle_mod):
    assert oracle_mod.grid_dim(1920, 1.0) == 1920
    assert oracle_mod.grid_dim(1920, 0.25) == 480
    assert oracle_mod.grid_dim(1080, 0.5) == 540
    assert oracle_mod.grid_dim(7, 0.25) == 2
    assert oracle_mod.grid_dim(1, 0.25) == 1
    for W in (7, 64, 1080, 1920):
        assert [oracle_mod.sample_pos(W, W, i) for i in range(W)] == list(range(W))
    # half resolution of an even width samples the odd pixels (centre of each pair)
    assert [oracle_mod.sample_pos(8, 4, i) for i in range(4)] == [1, 3, 5, 7]
    for W, Ws in ((1920, 480), (1080, 597), (13, 4)):
        s = [oracle_mod.sample_pos(W, Ws, i) for i in range(Ws)]
        assert s == sorted(s) and len(set(s)) == Ws and 0 <= s[0] and s[-1] < W
        # sample i lies inside its grid cell [i W / Ws, (i+1) W / Ws)
        for i, x in enumerate(s):
            assert i * W <= (x + 0.5) * Ws < (i + 1) * W


def test_upsample_identity_constant_ramp(oracle_mod):
    rng = np.random.default_rng(3)
    g = rng.random((9, 13, 2))
    np.testing.assert_array_equal(oracle_mod.upsample(g, 13, 9), g)  # s = 1
    c = np.full((5, 7, 1), 0.375)
    np.testing.assert_allclose(oracle_mod.upsample(c, 28, 20), 0.375, atol=1e-15)
    # a linear ramp over grid coordinates is reproduced in the interior
    Ws, Hs, W, H = 10, 6, 40, 24
    gx, gy = np.meshgrid(np.arange(Ws), np.arange(Hs))
    ramp = (0.3 * gx + 0.7 * gy)[:, :, None].astype(np.float64)
    up = oracle_mod.upsample(ramp, W, H)[:, :, 0]
    for y in range(H):
        for x in range(W):
            u = ((2 * x + 1) * Ws - W) / (2 * W)
            v = ((2 * y + 1) * Hs - H) / (2 * H)
            if 0 <= u <= Ws - 1 and 0 <= v <= Hs - 1:
                assert abs(up[y, x] - (0.3 * u + 0.7 * v)) < 1e-12


def test_learned_full_resolution_reduces_to_per_pixel(oracle_mod, sg):
    """At s2 = s3 = 1 the mixed-resolution path equals the per-pixel formula of
    eq (3) with the pixel's own layer 2 and tail features."""
    fr = sg.Scene("c1_256").frame(0)
    o = oracle_mod.frame_of(fr)
    Ws, bs = sg.init_mlp((16, 32, 32, 3), out_bias=0.05)
    mlp = oracle_mod.Mlp(Ws, bs)
    rgb, xf, f = oracle_mod.learned(o["lay"], o["tail"], fr.width, fr.height,
                                    (fr.width, fr.height, fr.width, fr.height), mlp)
    x = oracle_mod.features(o["lay"], o["tail"])
    np.testing.assert_array_equal(xf, x)
    y = mlp.forward(x)
    N = o["lay"][:, 0:1]
    y = np.where(N >= 3, y, 0.0)
    np.testing.assert_array_equal(f, y)
    L = o["lay"]
    a1, c1, a2, c2 = L[:, 2:3], L[:, 3:6], L[:, 6:7], L[:, 7:10]
    T2 = (1 - a1) * (1 - a2)
    tt = np.where(N >= 3, x[:, 1:2], 1.0)
    want = a1 * c1 + (1 - a1) * a2 * c2 + T2 * y + T2 * tt * 1.0
    np.testing.assert_allclose(rgb, want, atol=1e-12)


# ---------------------------------------------------------------------------
# eq (4) and the complexity index

def test_pass_scales_paper_facts(oracle_mod):
    """Sec. 3.2: s2 = 1 when wbar = 2.2, s3 = 1 when wbar = 3.0; both clamp at 0.25."""
    s2, s3 = oracle_mod.pass_scales(2.2)
    assert s2 == 1.0 and abs(s3 - 2 ** -0.8) < 1e-15
    assert oracle_mod.pass_scales(3.0) == (1.0, 1.0)
    assert oracle_mod.pass_scales(0.0) == (0.25, 0.25)
    s2, s3 = oracle_mod.pass_scales(1.2)
    assert abs(s2 - 0.5) < 1e-15 and abs(s3 - 2 ** -1.8) < 1e-15
    assert oracle_mod.pass_scales(0.9)[1] == 0.25  # 2^-2.1 < 0.25 clamps
    s2, s3 = oracle_mod.pass_scales(2.0)
    assert abs(s2 - 2 ** -0.2) < 1e-15 and abs(s3 - 0.5) < 1e-15
    # a unit increase of wbar doubles the unclamped scale
    a, _ = oracle_mod.pass_scales(0.7)
    b, _ = oracle_mod.pass_scales(1.7)
    assert abs(b / a - 2.0) < 1e-14


def test_wbar(oracle_mod):
    assert oracle_mod.wbar([0, 0, 0, 0]) == 0.0
    assert oracle_mod.wbar([5, 0, 0, 0]) == 0.0
    assert oracle_mod.wbar([0, 0, 0, 9]) == 3.0
    assert oracle_mod.wbar([1, 1, 1, 1]) == 1.5
    assert oracle_mod.wbar([3, 0, 1, 0]) == 0.5


def test_paper_golden_pass_scale_facts(oracle_mod):
    """Golden facts printed in the paper (tests/golden/pass_scales.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "pass_scales.txt")
    n = 0
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        wb, s2, s3 = [float(v) if v != "-" else None for v in line.split()]
        g2, g3 = oracle_mod.pass_scales(wb)
        if s2 is not None:
            assert abs(g2 - s2) < 1e-12
        if s3 is not None:
            assert abs(g3 - s3) < 1e-12
        n += 1
    assert n >= 3
