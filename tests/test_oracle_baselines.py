"""Pins of the oracle's cheap baselines (Sec. 4): weighted blended OIT with the
McGuire-Bavoil depth weight, and blending in stored order with no sort (the
paper's "random order" renderer behind E_random)."""
import numpy as np
import pytest

from csr_util import make_csr, random_lists


def _frame(lists, W, H):
    off, dep, rgba, prim = make_csr(lists, W, H)
    return off, dep, rgba, prim


@pytest.mark.parametrize("z,a,w", [
    (0.0, 1.0, 3000.0),    # (1 - z)^3 = 1
    (0.0, 0.2, 600.0),     # the weight carries a factor a
    (0.5, 1.0, 375.0),     # 3000 / 8
    (0.9, 1.0, 3.0),       # 3000 * 1e-3
    (0.99, 1.0, 1e-2),     # 3000 * 1e-6 = 3e-3 is below the floor
    (1.0, 0.5, 5e-3),      # floor 1e-2 times a
])
def test_wboit_weight_values(oracle_mod, z, a, w):
    """Values of the weight at hand-evaluated points."""
    assert oracle_mod.wboit_weight(z, a) == pytest.approx(w, rel=1e-12, abs=1e-15)


def test_wboit_two_fragments_closed_form(oracle_mod):
    """Red at z = 0 and blue at z = 0.5, both a = 1/2: weights 1500 and 187.5,
    weighted alphas 750 and 93.75 (ratio 8 : 1), revealage 1/4, so
    C = 3/4 (8/9 red + 1/9 blue) + 1/4 C_b, in either stored order."""
    bg = np.array([0.2, 0.4, 0.6])
    want = np.array([2 / 3, 0.0, 1 / 12]) + 0.25 * bg
    for order in ([(0.0, 1, 1, 0, 0, 0.5), (0.5, 2, 0, 0, 1, 0.5)],
                  [(0.5, 2, 0, 0, 1, 0.5), (0.0, 1, 1, 0, 0, 0.5)]):
        off, dep, rgba, _ = _frame([order], 1, 1)
        out = oracle_mod.baseline(off, dep, rgba, 1, 1, oracle_mod.BASE_WBOIT, bg)
        np.testing.assert_allclose(out[0], want, rtol=0, atol=1e-15)


def test_wboit_single_fragment_is_exact_over(oracle_mod):
    """With one fragment the weight cancels: C = a c + (1 - a) C_b, as the
    exact composite gives."""
    rng = np.random.default_rng(3)
    lists = random_lists(rng, 9, 7, 1)
    off, dep, rgba, prim = _frame(lists, 9, 7)
    bg = (0.1, 0.7, 0.3)
    out = oracle_mod.baseline(off, dep, rgba, 9, 7, oracle_mod.BASE_WBOIT, bg)
    ex = oracle_mod.frame(off, dep, rgba, prim, 9, 7, bg=bg, want=("rgb",))["rgb"]
    np.testing.assert_allclose(out, ex, rtol=0, atol=1e-14)


def test_wboit_uniform_colour_is_exact(oracle_mod):
    """Fragments that all share one colour c: whatever the weights,
    C = c (1 - prod(1 - a)) + prod(1 - a) C_b, the exact composite."""
    rng = np.random.default_rng(4)
    lists = random_lists(rng, 8, 8, 12)
    c = (0.25, 0.5, 0.75)
    lists = [[(z, pr, *c, a) for (z, pr, r, g, b, a) in l] for l in lists]
    off, dep, rgba, prim = _frame(lists, 8, 8)
    out = oracle_mod.baseline(off, dep, rgba, 8, 8, oracle_mod.BASE_WBOIT)
    ex = oracle_mod.frame(off, dep, rgba, prim, 8, 8, want=("rgb",))["rgb"]
    np.testing.assert_allclose(out, ex, rtol=0, atol=1e-13)


def test_wboit_is_order_independent(oracle_mod):
    """Reversing every list changes nothing beyond rounding."""
    rng = np.random.default_rng(5)
    lists = random_lists(rng, 8, 8, 20)
    off, dep, rgba, _ = _frame(lists, 8, 8)
    off2, dep2, rgba2, _ = _frame([l[::-1] for l in lists], 8, 8)
    a = oracle_mod.baseline(off, dep, rgba, 8, 8, oracle_mod.BASE_WBOIT)
    b = oracle_mod.baseline(off2, dep2, rgba2, 8, 8, oracle_mod.BASE_WBOIT)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


def test_over_list_on_sorted_lists_is_exact(oracle_mod):
    """Lists stored front to back: blending in stored order is the exact
    A-buffer composite."""
    rng = np.random.default_rng(6)
    lists = [sorted(l, key=lambda f: (f[0], f[1])) for l in random_lists(rng, 10, 6, 15)]
    off, dep, rgba, prim = _frame(lists, 10, 6)
    bg = (0.9, 0.1, 0.5)
    out = oracle_mod.baseline(off, dep, rgba, 10, 6, oracle_mod.BASE_OVER_LIST, bg)
    ex = oracle_mod.frame(off, dep, rgba, prim, 10, 6, bg=bg, want=("rgb",))["rgb"]
    np.testing.assert_allclose(out, ex, rtol=0, atol=1e-14)


def test_over_list_follows_stored_order(oracle_mod):
    """Two fragments blended as stored, back one first:
    C = a2 c2 + (1 - a2) a1 c1 + (1 - a1)(1 - a2) C_b."""
    f1 = (0.1, 1, 1.0, 0.0, 0.0, 0.5)   # front, red
    f2 = (0.9, 2, 0.0, 1.0, 0.0, 0.25)  # back, green, stored first
    off, dep, rgba, _ = _frame([[f2, f1]], 1, 1)
    bg = np.array([0.0, 0.0, 1.0])
    out = oracle_mod.baseline(off, dep, rgba, 1, 1, oracle_mod.BASE_OVER_LIST, bg)
    want = 0.25 * np.array([0, 1, 0]) + 0.75 * 0.5 * np.array([1, 0, 0]) + 0.5 * 0.75 * bg
    np.testing.assert_allclose(out[0], want, rtol=0, atol=1e-15)


def test_baselines_empty_pixels_and_unknown_method(oracle_mod):
    off, dep, rgba, _ = _frame([[], []], 2, 1)
    bg = (0.3, 0.2, 0.1)
    for m in (oracle_mod.BASE_WBOIT, oracle_mod.BASE_OVER_LIST):
        np.testing.assert_array_equal(oracle_mod.baseline(off, dep, rgba, 2, 1, m, bg), [bg, bg])
    with pytest.raises(ValueError):
        oracle_mod.baseline(off, dep, rgba, 2, 1, 7, bg)


def test_selective_inference_extremes(oracle_mod, sg):
    """All cells flat: the f_avg composite; no cell flat: the learned one."""
    fr = sg.Scene("c1_256", width=40, height=24, num_tris=20).frame(0)
    o = oracle_mod.frame_of(fr, want=("lay", "tail"))
    W, H = fr.width, fr.height
    grids = (W, H, W, H)
    Ws, bs = sg.init_mlp((16, 8, 8, 3), seed=2, out_bias=0.1)
    m = oracle_mod.Mlp(Ws, bs)
    cells = ((W + 7) // 8) * ((H + 7) // 8)
    learned, _, _ = oracle_mod.learned(o["lay"], o["tail"], W, H, grids, m)
    favg, _, _ = oracle_mod.learned(o["lay"], o["tail"], W, H, grids, None, oracle_mod.MODE_FAVG)
    np.testing.assert_array_equal(oracle_mod.selective(o["lay"], o["tail"], W, H, grids, m, np.zeros(cells), 64), favg)
    np.testing.assert_array_equal(oracle_mod.selective(o["lay"], o["tail"], W, H, grids, m, np.full(cells, 2), 64),
                                  learned)
    # only cell (1, 0) flat: exactly the pixels of columns 8..15, rows 0..7
    lv = np.full(cells, 3)
    lv[1] = 0
    out = oracle_mod.selective(o["lay"], o["tail"], W, H, grids, m, lv, 64).reshape(H, W, 3)
    np.testing.assert_array_equal(out[0:8, 8:16], favg.reshape(H, W, 3)[0:8, 8:16])
    mask = np.ones((H, W), bool)
    mask[0:8, 8:16] = False
    np.testing.assert_array_equal(out[mask], learned.reshape(H, W, 3)[mask])
