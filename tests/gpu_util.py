"""Helpers for GPU tests: run library calls on seeded frames and read results
back. Marshalling only; every computation happens in libstarnt."""
import numpy as np
import torch


def sync():
    torch.cuda.synchronize()


def run_features(st, fr, sched=None, max_per_pixel=None, with_sel=True):
    df = st.DeviceFrags.from_frame(fr, max_per_pixel=max_per_pixel)
    fb = st.FeatBuffers(fr.width, fr.height, with_sel=with_sel)
    st.starnt_features(df, sched, fb)
    sync()
    return df, fb


def to_np(t):
    return t.detach().cpu().numpy()


def sel_np(fb):
    return to_np(fb.sel).view(np.uint32)


def run_exact(st, df, bg=(1.0, 1.0, 1.0), feats=None):
    P = df.width * df.height
    rgb = torch.empty(P, 3, dtype=torch.float32, device="cuda")
    fstar = torch.empty(P, 3, dtype=torch.float32, device="cuda")
    st.starnt_composite(df, feats, None, None, bg, st.MODE_EXACT, rgb, fstar)
    sync()
    return to_np(rgb), to_np(fstar)


def run_learned(st, df, fb, mlp, sched, bg=(1.0, 1.0, 1.0), mode=None):
    P = df.width * df.height
    mode = st.MODE_LEARNED if mode is None else mode
    tail_rgb = torch.zeros(P, 3, dtype=torch.float32, device="cuda")
    if mode == st.MODE_LEARNED:
        st.starnt_infer(mlp, fb.tail, fb.count, sched, df.width, df.height, tail_rgb)
    rgb = torch.empty(P, 3, dtype=torch.float32, device="cuda")
    st.starnt_composite(df, fb, tail_rgb, sched, bg, mode, rgb)
    sync()
    return to_np(rgb), to_np(tail_rgb)
