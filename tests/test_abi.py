"""The C-ABI library loads and exports every call the header declares; host
helpers and host-side validation work without a GPU (no kernel is launched)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "starnt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(starnt_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_six_calls():
    names = header_functions()
    for n in ("starnt_features", "starnt_infer", "starnt_composite", "starnt_quadtree", "starnt_reproject",
              "starnt_train_step"):
        assert n in names


def test_library_exports_every_declared_symbol(starnt):
    lib = ctypes.CDLL(starnt.LIB_PATH)
    for n in header_functions():
        assert hasattr(lib, n), n
    assert set(header_functions()) == set(starnt.EXPORTS)
    assert starnt.starnt_version().startswith("starnt")


def test_host_helpers_match_the_pinned_oracle(starnt, oracle_mod):
    for wb in (0.0, 0.2, 0.7, 1.2, 2.0, 2.2, 2.9, 3.0):
        a = starnt.starnt_pass_scales(wb)
        b = oracle_mod.pass_scales(wb)
        assert abs(a[0] - b[0]) < 1e-15 and abs(a[1] - b[1]) < 1e-15
    for h in ([0, 0, 0, 0], [1, 1, 1, 1], [3, 0, 1, 0], [0, 5, 0, 7]):
        assert starnt.starnt_wbar(h) == oracle_mod.wbar(h)
    for n in (1, 7, 1080, 1920):
        for s in (0.25, 0.3, 0.5, 0.77, 1.0):
            assert starnt.starnt_grid_dim(n, s) == oracle_mod.grid_dim(n, s)


def test_m_minus_i_helper_matches_the_oracle(starnt, oracle_mod, sg):
    """The library's host helper for the reprojection matrix equals the
    oracle's M - I (both FP64, rounded to FP32) on the camera path of the
    1080p workload and on a random well-conditioned pair; a singular current
    matrix is rejected."""
    sc = sg.Scene("c2_1080p", width=64, height=36, num_tris=10)
    rng = np.random.default_rng(0)
    pairs = [(sc.camera(0), sc.camera(t)) for t in range(1, 8)]
    pairs.append((rng.normal(size=(4, 4)) + 4 * np.eye(4), rng.normal(size=(4, 4)) + 4 * np.eye(4)))
    for a, b in pairs:
        got = starnt.starnt_m_minus_i(a, b)
        want = oracle_mod.m_minus_i(a, b)
        assert np.abs(got.astype(np.float64) - want).max() <= 1e-6 * max(1.0, np.abs(want).max())
    with pytest.raises(starnt.StarntError):
        starnt.starnt_m_minus_i(np.eye(4), np.zeros((4, 4)))


def test_workspace_sizes(starnt):
    assert starnt.starnt_workspace_size(starnt.WS_QUADTREE, 1920, 1080, 64) > 0
    assert starnt.starnt_workspace_size(starnt.WS_QUADTREE, 1920, 1080, 12) == 0  # not a multiple of 8
    n = starnt.starnt_workspace_size(starnt.WS_TRAIN, 65536, 64, 64)
    params = 64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3
    assert n >= 1024 * params * 4
    assert starnt.starnt_workspace_size(99, 1, 1, 1) == 0


def test_error_word_mapping(starnt):
    starnt.starnt_check(0)
    for w in (1, 2, 4, 7):
        with pytest.raises(starnt.StarntError) as e:
            starnt.starnt_check(w)
        assert e.value.code == 2


def test_host_validation_rejects_bad_arguments(starnt):
    """Invalid arguments are refused on the host with EINVAL/ENOMEM before any
    launch (NULL pointers are never dereferenced on the device)."""
    lib = starnt.lib
    fr = starnt.Frags(0, 0, None, None, None, 0, None, 0, 1)
    ft = starnt.Feats(0, 0, None, None, None, None, None, None, None)
    assert lib.starnt_features(ctypes.byref(fr), None, ctypes.byref(ft), None) == 1
    fr = starnt.Frags(64, 64, 16, 16, 16, 7, 16, 10, 1)  # bad rgba dtype (pointers never used)
    assert lib.starnt_features(ctypes.byref(fr), None, ctypes.byref(ft), None) == 1
    assert b"rgba_dtype" in lib.starnt_last_error()
    assert lib.starnt_features(None, None, None, None) == 1
    qp = starnt.QtParams(12, 0.1, 0.05, 2)
    assert lib.starnt_quadtree(16, 16, 64, 64, ctypes.byref(qp), None, 16, 16, 16, 16, 1 << 20, None) == 1
    qp = starnt.QtParams(64, 0.1, 0.05, 2)
    assert lib.starnt_quadtree(16, 16, 64, 64, ctypes.byref(qp), None, 16, 16, 16, 16, 10, None) == 3
    qp = starnt.QtParams(64, 0.05, 0.1, 2)  # merge above split
    assert lib.starnt_quadtree(16, 16, 64, 64, ctypes.byref(qp), None, 16, 16, 16, 16, 1 << 20, None) == 1
    m = (ctypes.c_float * 16)(*([0.0] * 15 + [float("nan")]))
    assert lib.starnt_reproject(1 << 20, 2 << 20, 8, 8, m, 3 << 20, None, None) == 1
    assert b"non-finite" in lib.starnt_last_error()
    mlp = starnt.Mlp(5, 32, 32, 3, 0, 16, 16, 16, 16, 16, 16, None)  # in must be 16
    assert lib.starnt_infer(ctypes.byref(mlp), 16, 16, None, 8, 8, 16, None) == 1
    mlp = starnt.Mlp(16, 32, 32, 3, 3, 16, 16, 16, 16, 16, 16, None)  # FP8 without scales
    assert lib.starnt_infer(ctypes.byref(mlp), 16, 16, None, 8, 8, 16, None) == 1
    tr = starnt.Train(16, 64, 64, 3, 0, 16, 16, 16, 16)
    ad = starnt.Adam(1e-3, 0.9, 0.999, 1e-8, 0)  # step must be >= 1
    assert lib.starnt_train_step(ctypes.byref(tr), 16, 16, 64, ctypes.byref(ad), 16, 16, 1 << 30, None) == 1
    ad = starnt.Adam(1e-3, 0.9, 0.999, 1e-8, 1)
    assert lib.starnt_train_step(ctypes.byref(tr), 16, 16, 64, ctypes.byref(ad), 16, 16, 8, None) == 3
    bg = (ctypes.c_float * 3)(1.0, 1.0, 1.0)
    assert lib.starnt_composite(None, None, None, None, bg, 9, 16, None, None) == 1
    fr = starnt.Frags(8, 8, 16, 16, 16, 0, None, 10, 1)
    assert lib.starnt_baseline(ctypes.byref(fr), 5, bg, 16, None) == 1  # unknown method
    assert b"method" in lib.starnt_last_error()
    assert lib.starnt_baseline(ctypes.byref(fr), 0, bg, None, None) == 1
    assert lib.starnt_baseline(None, 0, bg, 16, None) == 1
    m = (ctypes.c_float * 16)(*([0.0] * 16))
    rc = lib.starnt_reproject_check
    rc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                   ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    need = starnt.starnt_workspace_size(starnt.WS_REPROJECT, 8, 8)
    assert need >= 8 + 2 * 4
    # fake device addresses (never dereferenced): rgb [64][3], d1 [64], out
    # [64][3] in disjoint ranges
    RGB, D1, OUT = 1 << 20, 2 << 20, 3 << 20
    assert rc(RGB, D1, 8, 8, m, -0.5, OUT, None, 64, 80, 256, need, None) == 1  # negative tolerance
    assert b"depth_tol" in lib.starnt_last_error()
    assert rc(RGB, D1, 8, 8, m, float("inf"), OUT, None, 64, 80, 256, need, None) == 1
    assert rc(RGB, D1, 8, 8, m, 0.01, OUT, None, None, 80, 256, need, None) == 1  # no list
    assert rc(RGB, D1, 8, 8, m, 0.01, RGB, None, 64, 80, 256, need, None) == 1    # output aliases input
    assert b"overlaps" in lib.starnt_last_error()
    assert rc(RGB, D1, 8, 8, m, 0.01, RGB + 764, None, 64, 80, 256, need, None) == 1  # last float shared
    assert rc(RGB, D1, 8, 8, m, 0.01, D1 - 767, None, 64, 80, 256, need, None) == 1   # first d1 byte shared
    assert rc(RGB, D1, 8, 8, m, 0.01, OUT, None, 64, 80, 256, need - 1, None) == 3  # workspace too small
    assert rc(RGB, D1, 8, 8, m, 0.01, OUT, None, 64, 80, 272, need, None) == 1      # misaligned workspace
    assert b"aligned" in lib.starnt_last_error()
    assert rc(RGB, D1, 8, 8, m, 0.01, OUT, None, 64, 80, None, need, None) == 1
    # an output right after the colour range and right before d1 overlaps nothing
    assert rc(RGB, D1, 8, 8, m, -1.0, RGB + 768, None, 64, 80, 256, need, None) == 1
    assert b"depth_tol" in lib.starnt_last_error()
    assert rc(RGB, D1, 8, 8, m, -1.0, D1 - 768, None, 64, 80, 256, need, None) == 1
    assert b"depth_tol" in lib.starnt_last_error()
    rp = lib.starnt_reproject
    rp.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert rp(RGB, D1, 8, 8, m, D1 + 100, None, None) == 1
    assert b"overlaps" in lib.starnt_last_error()
    fr = starnt.Frags(8, 8, 16, 16, 16, 0, 16, 10, 1)
    slots = starnt.Feats(4, 1, 16, 16, 16, 16, 16, None, 16, None)
    mlp = starnt.Mlp(16, 32, 32, 3, 0, 16, 16, 16, 16, 16, 16, None)
    patch = lib.starnt_patch
    bad = starnt.Feats(4, 2, 16, 16, 16, 16, 16, None, 16, None)  # slots must be one row
    assert patch(ctypes.byref(fr), ctypes.byref(mlp), 16, 16, ctypes.byref(bad), bg, 16, None) == 1
    assert b"1-row" in lib.starnt_last_error()
    assert patch(ctypes.byref(fr), ctypes.byref(mlp), None, 16, ctypes.byref(slots), bg, 16, None) == 1
    dfa = starnt.Mlp(16, 32, 32, 3, 0, 16, 16, 16, 16, 16, 16, None, 1)
    assert patch(ctypes.byref(fr), ctypes.byref(dfa), 16, 16, ctypes.byref(slots), bg, 16, None) == 5


def test_product_package_has_no_cpu_fallback():
    """The product package never imports the oracle or a CPU path."""
    pkg = os.path.join(ROOT, "paper_2606_16747_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "oracle.c" not in txt, f


def test_time_next_launch_request_without_events(starnt):
    """A request with no events is accepted and clears any pending one; it
    touches no GPU state, so it runs without a device."""
    starnt.starnt_time_next_launch(None, None)
    assert starnt.lib.starnt_time_next_launch(None, None) == 0  # STARNT_OK
