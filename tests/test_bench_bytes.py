"""The bench's algorithmic byte counts, which its rooflines divide by measured
times, on a hand-built two-pixel frame (values worked out by hand below)."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_for_tests", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _Frame:
    """Two pixels in one row with 3 and 1 fragments, FP32 RGBA."""
    width, height, num_frags = 2, 1, 4
    rgba = np.zeros((4, 4), np.float32)

    def counts(self):
        return np.array([3, 1], np.int64)


def test_sample_positions(bench):
    # sample i of ns sits at floor((2i + 1) n / (2 ns))
    assert bench.sample_mask(7, 7).all()
    m = bench.sample_mask(8, 1)
    assert m.sum() == 1 and m[4]
    assert np.flatnonzero(bench.sample_mask(10, 4)).tolist() == [1, 3, 6, 8]


def test_fragment_pass_bytes_full_resolution(bench):
    # reads: offsets 4 * 3, depths 4 * 4, RGBA of every fragment 16 * 4 = 92;
    # writes: 24 per pixel, 16 per pass-2 and 32 per pass-3 sample = 144
    total, streamed = bench.feature_pass_bytes(_Frame(), (2, 1, 2, 1))
    assert (total, streamed) == (236, 4)


def test_fragment_pass_bytes_one_pass3_sample(bench):
    # the one pass-3 sample is pixel 1 (1 fragment): reads 12 + 16 + 16 (its
    # RGBA) + 16 (layer-1 gather of pixel 0) + 16 (its layer-2 gather: N = 3
    # and a pass-2 sample) = 76; writes 48 + 32 + 32 = 112
    total, streamed = bench.feature_pass_bytes(_Frame(), (2, 1, 1, 1))
    assert (total, streamed) == (188, 1)


def test_inference_bytes(bench):
    # 32 B per pixel, 16 per pass-2 sample, 32 per pass-3 record
    assert bench.infer_pass_bytes(2, 1, (2, 1, 1, 1)) == 32 * 2 + 16 * 2 + 32


def _trace(rows, col="grid_size_x"):
    """An in-memory kernel trace: rows of (dispatch_id, name, grid)."""
    import sqlite3
    con = sqlite3.connect(":memory:")
    con.execute("create table kernels (dispatch_id integer, name text, start integer, duration integer, %s integer)"
                % col)
    con.executemany("insert into kernels values (?, ?, 0, 0, ?)", rows)
    return con


def test_exact_launches_picked_by_frame_size(bench):
    """The profile summary averages the exact kernel over the 1080p frames
    only: launches of the same variant on smaller frames (the training
    scenes) and of other variants are left out, whichever unit the trace
    gives the grid in."""
    pat = "WaveCfg<192, 16>, false, false>"
    name = "void starnt::exact_wave_kernel<starnt::WaveCfg<192, 16>, false, false>(starnt::ExactArgs)"
    other = "void starnt::exact_wave_kernel<starnt::WaveCfg<192, 16>, false, true>(starnt::ExactArgs)"
    P = 1920 * 1080
    small = 480 * 270
    rows = [(1, name, small // 16 * 64), (2, other, P // 16 * 64), (3, name, P // 16 * 64),
            (4, name, small // 16 * 64), (5, name, P // 16 * 64)]
    # positions among the variant's own launches in dispatch order: 0, 1, 2, 3
    assert bench.exact_launches_of_frame(_trace(rows), pat, P) == [1, 3]
    wg = [(d, n, g // 64) for d, n, g in rows]
    assert bench.exact_launches_of_frame(_trace(wg, "grid_x"), pat, P) == [1, 3]
    with pytest.raises(SystemExit):
        bench.exact_launches_of_frame(_trace(rows), pat, 2560 * 1440)
    with pytest.raises(SystemExit):
        bench.exact_launches_of_frame(_trace(rows, "workgroups"), pat, P)
