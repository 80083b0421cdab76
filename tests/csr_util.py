"""Hand-built fragment lists for small tests (plain data, no method arithmetic)."""
import numpy as np


def make_csr(lists, width, height):
    """lists[p] = [(z, prim, r, g, b, a), ...] -> (offsets, depth, rgba, prim)."""
    P = width * height
    assert len(lists) == P
    counts = [len(l) for l in lists]
    offsets = np.zeros(P + 1, np.uint32)
    offsets[1:] = np.cumsum(counts)
    F = int(offsets[-1])
    depth = np.zeros(F, np.float32)
    rgba = np.zeros((F, 4), np.float32)
    prim = np.zeros(F, np.uint32)
    k = 0
    for l in lists:
        for (z, pr, r, g, b, a) in l:
            depth[k] = z
            prim[k] = pr
            rgba[k] = (r, g, b, a)
            k += 1
    return offsets, depth, rgba, prim


def random_lists(rng, width, height, max_n, ties=False):
    """Random per-pixel lists with unique (depth, prim) keys; with ties=True
    depths are drawn from a tiny set so equal depths are common."""
    lists = []
    for _ in range(width * height):
        n = int(rng.integers(0, max_n + 1))
        prims = rng.choice(10 * max_n + 10, size=n, replace=False)
        if ties:
            zs = rng.choice(np.array([0.0, 0.25, 0.5, 0.75, 1.0], np.float32), size=n)
        else:
            zs = rng.random(n).astype(np.float32)
        l = []
        for z, pr in zip(zs, prims):
            r, g, b = rng.random(3)
            a = float(rng.uniform(0.05, 0.95))
            l.append((float(z), int(pr), float(r), float(g), float(b), a))
        lists.append(l)
    return lists


def sub_csr(offsets, depth, rgba, prim, pixels):
    """The lists of the given pixels, in that order, as the CSR arrays of a
    1 x len(pixels) frame (plain slicing; rgba keeps its dtype)."""
    offsets = np.asarray(offsets, np.int64)
    pixels = np.asarray(pixels, np.int64)
    b, e = offsets[pixels], offsets[pixels + 1]
    counts = e - b
    sub_off = np.zeros(len(pixels) + 1, np.uint32)
    sub_off[1:] = np.cumsum(counts)
    idx = np.concatenate([np.arange(x, y) for x, y in zip(b, e)]) if len(pixels) else np.zeros(0, np.int64)
    idx = idx.astype(np.int64)
    return sub_off, depth[idx], rgba[idx], prim[idx], idx
