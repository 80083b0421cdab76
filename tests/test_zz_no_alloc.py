"""The allocation-free quadtree update (starnt_quadtree_noalloc) against
starnt_quadtree with a caller workspace, through the C ABI: masks, levels and
the device schedule bitwise equal, over two frames chained through the
previous mask, on a 1920x1080 frame and then on a smaller 400x224 one (the
library's fixed scratch keeps the larger call's contents)."""
import numpy as np
import pytest
import torch

from gpu_util import run_exact, sync, to_np

pytestmark = pytest.mark.gpu


def _inputs(starnt, sg, W, H, t):
    sc = sg.Scene("c2_1080p", width=W, height=H, num_tris=max(200, W * H // 1000))
    df = starnt.DeviceFrags.from_frame(sc.frame(t), max_per_pixel=64)
    rgb, _ = run_exact(starnt, df)
    fb = starnt.FeatBuffers(W, H)
    starnt.starnt_features(df, None, fb)
    sync()
    return torch.from_numpy(rgb).cuda(), fb.count


@pytest.mark.parametrize("k_relax", [2, 1])
def test_quadtree_noalloc_equals_workspace_call(starnt, gpu, sg, k_relax):
    qp = starnt.QtParams(64, 0.10, 0.05, k_relax)
    for W, H in ((1920, 1080), (400, 224)):
        T = ((W + 63) // 64) * ((H + 63) // 64)
        C = ((W + 7) // 8) * ((H + 7) // 8)
        ws = starnt.workspace(starnt.starnt_workspace_size(starnt.WS_QUADTREE, W, H, 64))
        out = {}
        for kind in ("ws", "noalloc"):
            masks = [torch.full((T,), -1, dtype=torch.int32, device="cuda") for _ in range(2)]
            level = torch.full((C,), 255, dtype=torch.uint8, device="cuda")
            sched = starnt.new_sched(W, H)
            prev = None
            res = []
            for t in range(2):
                rgb, count = _inputs(starnt, sg, W, H, t)
                cur = masks[t % 2]
                if kind == "ws":
                    starnt.starnt_quadtree(rgb, count, W, H, qp, prev, cur, level, sched, ws)
                else:
                    starnt.starnt_quadtree_noalloc(rgb, count, W, H, qp, prev, cur, level, sched)
                sync()
                res.append((to_np(cur).copy(), to_np(level).copy(), to_np(sched).copy()))
                prev = cur
            out[kind] = res
        for (m0, l0, s0), (m1, l1, s1) in zip(out["ws"], out["noalloc"]):
            assert np.array_equal(m0, m1) and np.array_equal(l0, l1) and np.array_equal(s0, s1)
        assert (out["ws"][1][0] != 0).any()  # something split


def test_quadtree_noalloc_rejects_frames_beyond_its_scratch(starnt, gpu):
    W, H = 16384, 16384  # base 8: one cell per pixel, far above 4 MiB of scratch
    qp = starnt.QtParams(8, 0.10, 0.05, 2)
    rgb = torch.zeros(1, 3, dtype=torch.float32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    mask = torch.zeros(1, dtype=torch.int32, device="cuda")
    level = torch.zeros(1, dtype=torch.uint8, device="cuda")
    sched = starnt.new_sched(64, 64)
    with pytest.raises(starnt.StarntError) as ei:
        starnt.starnt_quadtree_noalloc(rgb, count, W, H, qp, None, mask, level, sched)
    assert ei.value.code == starnt.ENOMEM and "scratch" in str(ei.value)
