"""Exact A-buffer path against the FP64 oracle at the shapes its kernels
split on: 16-pixel waves whose batches hold 192, 256 or 384 fragments (the
smallest that holds the declared maximum list length; longer lists go to
the long-list kernel), lists at and around each capacity, runs of long lists
next to short ones, equal depths inside short and long lists, waves whose
pixels are all empty, and the call without the tail output. Bar: <= 1e-4 per channel against FP64 (eq (1), the A-buffer of
Sec. 4); the colour is bitwise the same with and without the tail output
and under permutation of every list."""
import numpy as np
import pytest
import torch

from csr_util import make_csr
from gpu_util import run_exact, sync, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _lists(rng, lengths, ties_every=0):
    lists = []
    for n in lengths:
        n = int(n)
        if ties_every and n > 1:
            # depths drawn from a small set: many equal depths in the list
            z = rng.integers(0, max(2, n // ties_every), size=n).astype(np.float32) / max(2, n // ties_every)
        else:
            z = rng.permutation(n).astype(np.float32) / max(n, 1)
        prims = rng.permutation(4 * n + 4)[:n]
        lists.append([(float(z[k]), int(prims[k]), *rng.random(3), float(rng.uniform(0.01, 0.3)))
                      for k in range(n)])
    return lists


def _check(starnt, oracle_mod, lists, W, H, max_n, bg=(0.3, 0.6, 0.9)):
    csr = make_csr(lists, W, H)
    df = starnt.DeviceFrags(*csr, W, H, max_n)
    rgb, fstar = run_exact(starnt, df, bg=bg)
    o = oracle_mod.frame(*csr, W, H, bg=bg)
    assert np.abs(rgb - o["rgb"]).max() <= TOL
    assert np.abs(fstar - o["fstar"]).max() <= TOL
    # the colour alone (no tail output) is the same colour, bit for bit
    P = W * H
    rgb_only = torch.empty(P, 3, dtype=torch.float32, device="cuda")
    starnt.starnt_composite(df, None, None, None, bg, starnt.MODE_EXACT, rgb_only, None)
    sync()
    assert np.array_equal(to_np(rgb_only), rgb)
    return csr, rgb, fstar


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_lists_around_the_batch_capacity(starnt, gpu, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    W, H = 64, 3
    lengths = rng.choice([0, 1, 2, 5, 17, 63, 200], size=W * H)
    # a wave of 64 pixels: lists at, below and above the batch capacity, a
    # run of long lists, a long list first and last in the wave
    lengths[0] = 385
    lengths[3:6] = (383, 384, 385)
    lengths[10:13] = (600, 700, 385)
    lengths[63] = 1000
    lengths[64 + 7] = 384
    lengths[64 + 8] = 384
    lengths[128:192] = 0  # four waves of empty pixels
    _check(starnt, oracle_mod, _lists(rng, lengths), W, H, 1024)


SPANNING = [
    (192, (10, 130, 52)),          # list 1 covers slots 64..127: no list starts there
    (192, (0, 60, 0, 8, 0, 120)),  # empty lists before, between and after; starts at 60 and 68
    (192, (1, 1, 190)),            # one list over all three blocks of 64 slots
    (384, (5, 300, 70, 9)),        # blocks 1..4 hold no start
    (384, (63, 1, 64, 1, 255)),    # starts at 63, 64, 128 and 129
]


@pytest.mark.parametrize("max_n,lengths", SPANNING)
def test_exact_lists_spanning_slot_blocks(starnt, gpu, oracle_mod, max_n, lengths):
    """Every fragment takes its list from a prefix maximum over the batch's
    slots, 64 slots at a time: lists that start right at and right after a
    block edge, and blocks inside one list (the maximum carried from earlier
    blocks alone names the list). One 16-pixel wave per case; the remaining
    pixels of the wave are empty."""
    rng = np.random.default_rng(sum(lengths))
    W, H = 16, 1
    full = list(lengths) + [0] * (W * H - len(lengths))
    _check(starnt, oracle_mod, _lists(rng, full), W, H, max_n)


@pytest.mark.parametrize("max_n,lengths", SPANNING)
def test_exact_lists_spanning_slot_blocks_half_with_ties(starnt, gpu, oracle_mod, max_n, lengths):
    """The same batches with FP16 RGBA and many equal depths in every list:
    the recount on (depth, primitive id) takes each fragment's list from the
    same prefix maximum."""
    rng = np.random.default_rng(100 + sum(lengths))
    W, H = 16, 1
    full = list(lengths) + [0] * (W * H - len(lengths))
    off, dep, rgba, prim = make_csr(_lists(rng, full, ties_every=4), W, H)
    h = rgba.astype(np.float16)
    df = starnt.DeviceFrags(off, dep, h, prim, W, H, max_n)
    bg = (0.5, 0.25, 0.75)
    rgb, fstar = run_exact(starnt, df, bg=bg)
    o = oracle_mod.frame(off, dep, h.astype(np.float32), prim, W, H, bg=bg)
    assert np.abs(rgb - o["rgb"]).max() <= TOL
    assert np.abs(fstar - o["fstar"]).max() <= TOL


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_small_batches_around_their_capacity(starnt, gpu, oracle_mod, seed):
    """Declared maximum 192: batches of at most 192 fragments. Lists at and
    below the capacity, waves whose lists need several batches, waves of
    empty pixels, a frame that is not a whole number of waves."""
    rng = np.random.default_rng(20 + seed)
    W, H = 61, 3
    lengths = rng.choice([0, 1, 2, 3, 9, 40, 96, 150], size=W * H)
    lengths[0] = 192
    lengths[1:4] = (191, 192, 1)
    lengths[15] = 192  # last pixel of the first wave
    lengths[32:64] = 0  # two waves of empty pixels
    lengths[64:70] = (100, 100, 100, 100, 100, 100)  # one list per batch
    lengths[-1] = 192
    _check(starnt, oracle_mod, _lists(rng, lengths), W, H, 192)


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_mid_batches_around_their_capacity(starnt, gpu, oracle_mod, seed):
    """Declared maximum 256: batches of at most 256 fragments, lists at, just
    below and well below that, one list per batch in a run, ties."""
    rng = np.random.default_rng(40 + seed)
    W, H = 50, 2
    lengths = rng.choice([0, 1, 7, 30, 129, 200], size=W * H)
    lengths[0:4] = (256, 255, 193, 256)
    lengths[16:32] = 0
    lengths[-1] = 256
    _check(starnt, oracle_mod, _lists(rng, lengths, ties_every=5 if seed else 0), W, H, 256)


def test_exact_small_batches_with_ties(starnt, gpu, oracle_mod):
    """The recount on (depth, prim) in the small configuration, and the same
    outputs under permutation of every list."""
    rng = np.random.default_rng(9)
    W, H = 45, 2
    lengths = rng.choice([0, 2, 5, 17, 64, 180], size=W * H)
    lists = _lists(rng, lengths, ties_every=3)
    csr, rgb, fstar = _check(starnt, oracle_mod, lists, W, H, 192)
    perm = [[l[k] for k in rng.permutation(len(l))] for l in lists]
    df2 = starnt.DeviceFrags(*make_csr(perm, W, H), W, H, 192)
    rgb2, fstar2 = run_exact(starnt, df2, bg=(0.3, 0.6, 0.9))
    assert np.array_equal(rgb, rgb2) and np.array_equal(fstar, fstar2)


@pytest.mark.parametrize("max_n", [192, 384])
def test_exact_half_colour(starnt, gpu, oracle_mod, max_n):
    """FP16 RGBA in the small and large configurations: the kernels convert
    each colour once; the oracle takes the same half values as FP32."""
    rng = np.random.default_rng(60 + max_n)
    W, H = 37, 3
    lengths = rng.choice([0, 1, 3, 8, 25, 90], size=W * H)
    lengths[0:3] = (max_n, max_n - 1, 2)
    off, dep, rgba, prim = make_csr(_lists(rng, lengths, ties_every=6), W, H)
    h = rgba.astype(np.float16)
    df = starnt.DeviceFrags(off, dep, h, prim, W, H, max_n)
    bg = (0.2, 0.4, 0.6)
    rgb, fstar = run_exact(starnt, df, bg=bg)
    o = oracle_mod.frame(off, dep, h.astype(np.float32), prim, W, H, bg=bg)
    assert np.abs(rgb - o["rgb"]).max() <= TOL
    assert np.abs(fstar - o["fstar"]).max() <= TOL


def test_exact_ties_in_short_and_long_lists(starnt, gpu, oracle_mod):
    rng = np.random.default_rng(5)
    W, H = 40, 4
    lengths = rng.choice([0, 3, 9, 30, 90], size=W * H)
    lengths[7] = 500
    lengths[50] = 384
    lists = _lists(rng, lengths, ties_every=4)
    csr, rgb, fstar = _check(starnt, oracle_mod, lists, W, H, 512)
    # permuting every list leaves both outputs bitwise unchanged
    perm = []
    for l in lists:
        idx = rng.permutation(len(l))
        perm.append([l[k] for k in idx])
    csr2 = make_csr(perm, W, H)
    df2 = starnt.DeviceFrags(*csr2, W, H, 512)
    rgb2, fstar2 = run_exact(starnt, df2, bg=(0.3, 0.6, 0.9))
    assert np.array_equal(rgb, rgb2) and np.array_equal(fstar, fstar2)


def test_exact_declared_maximum_below_the_capacity(starnt, gpu, oracle_mod):
    """With every list at most 384 long only the per-wave kernel runs; a frame
    wider than one wave with ragged tails (P not a multiple of 64)."""
    rng = np.random.default_rng(11)
    W, H = 97, 5
    lengths = rng.choice([0, 1, 4, 8, 32, 120, 384], size=W * H)
    _check(starnt, oracle_mod, _lists(rng, lengths), W, H, 384)


def test_exact_flags_lists_longer_than_declared(starnt, gpu):
    """A list longer than the declared maximum sets the count flag (the call
    itself is not an error; the flag is read after the stream), and every
    pixel is still written."""
    rng = np.random.default_rng(2)
    W, H = 8, 1
    lengths = [3, 400, 2, 0, 5, 6, 7, 8]
    lists = _lists(rng, lengths)
    csr = make_csr(lists, W, H)
    df = starnt.DeviceFrags(*csr, W, H, 64)
    fb = starnt.FeatBuffers(W, H)
    rgb = torch.full((W * H, 3), float("nan"), dtype=torch.float32, device="cuda")
    fb.err.zero_()
    starnt.starnt_composite(df, fb, None, None, (1, 1, 1), starnt.MODE_EXACT, rgb, None)
    sync()
    e = int(to_np(fb.err)[0])
    assert e & starnt.DERR_COUNT
    # every pixel is written: the list past every batch size gets the
    # background alone, the others their exact colour
    out = to_np(rgb)
    assert np.isfinite(out).all()
    assert np.array_equal(out[1], np.ones(3, np.float32))
