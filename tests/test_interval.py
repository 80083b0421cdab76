"""Adaptive interpolation interval (Sec. 3.3): pins of the oracle's policy on
hand-traced sequences, then the library's host implementation against the
oracle on seeded random cost sequences (decisions identical)."""
import numpy as np
import pytest


def _kinds(s):
    return "".join("R" if k else "I" for k in s)


@pytest.mark.parametrize("real,interp,target,maxk,want", [
    (10.0, 1.0, 16.7, 4, "RRRRRRRRRR"),          # real frames meet the target alone
    (30.0, 2.0, 16.7, 4, "RRIRIRIRIR"),          # probe, then (30 + 2) / 2 = 16 <= 16.7
    (50.0, 2.0, 16.7, 4, "RRIRIIIRII"),          # 26, 18 too slow; (50 + 6) / 4 = 14
    (100.0, 2.0, 16.7, 4, "RRIRRRRRRR"),         # (100 + 6) / 4 = 26.5: back to all real
    (50.0, 2.0, 16.7, 3, "RRIRRRRRRR"),          # the longest interval 3 gives 18
    (30.0, 2.0, 16.7, 1, "RRRRRRRRRR"),          # interpolation switched off
    (30.0, 20.0, 16.7, 4, "RRIRRRRRRR"),         # interpolation too dear to help
])
def test_policy_hand_traced(oracle_mod, real, interp, target, maxk, want):
    kinds, _ = oracle_mod.interval_schedule([(real, interp)] * len(want), target, maxk, 0.5)
    assert _kinds(kinds) == want


def test_policy_running_means(oracle_mod):
    """Means move by smoothing * (sample - mean) from the first sample:
    real samples 10, 20, 40 with smoothing 1/2 give 10 -> 15 -> 27.5."""
    kinds, (r, i) = oracle_mod.interval_schedule([(10.0, 1.0), (20.0, 1.0), (40.0, 1.0)], 50.0, 4, 0.5)
    assert kinds == [True, True, True] and r == 27.5 and i is None


def test_policy_adapts_to_a_slowdown(oracle_mod):
    """A scene that becomes heavy: first all real, then interpolation starts
    (after the probe) once the real cost passes the target."""
    costs = [(10.0, 1.0)] * 4 + [(40.0, 1.0)] * 8
    kinds, _ = oracle_mod.interval_schedule(costs, 16.7, 4, 1.0)
    assert _kinds(kinds) == "RRRR" + "RRIRIIRIIRII"[:8]


def test_library_matches_oracle_on_random_sequences(starnt, oracle_mod):
    rng = np.random.default_rng(3)
    for trial in range(40):
        n = int(rng.integers(1, 60))
        base_r, base_i = rng.uniform(2, 80), rng.uniform(0.2, 10)
        costs = [(float(base_r * rng.uniform(0.7, 1.3)), float(base_i * rng.uniform(0.7, 1.3))) for _ in range(n)]
        target = float(rng.uniform(5, 40))
        maxk = int(rng.integers(1, 5))
        sm = float(rng.uniform(0.05, 1.0))
        want, means = oracle_mod.interval_schedule(costs, target, maxk, sm)
        s = starnt.starnt_interval_init(target, maxk, sm)
        got = []
        for t in range(n):
            real = starnt.starnt_interval_next(s)
            got.append(real)
            starnt.starnt_interval_report(s, real, costs[t][0 if real else 1])
        assert got == want, (trial, _kinds(got), _kinds(want))
        assert s.real_ms == pytest.approx(means[0] if means[0] is not None else -1.0, rel=1e-12)


def test_library_rejects_bad_arguments(starnt):
    with pytest.raises(starnt.StarntError):
        starnt.starnt_interval_init(0.0)
    with pytest.raises(starnt.StarntError):
        starnt.starnt_interval_init(16.7, 5)
    with pytest.raises(starnt.StarntError):
        starnt.starnt_interval_init(16.7, 4, 0.0)
    s = starnt.starnt_interval_init(16.7)
    with pytest.raises(starnt.StarntError):
        starnt.starnt_interval_report(s, True, float("nan"))
    with pytest.raises(starnt.StarntError):
        starnt.starnt_interval_report(s, True, -1.0)
