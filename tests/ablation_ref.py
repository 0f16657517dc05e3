"""The ablation of Sec. 5.3's design choices computed with the FP64 oracle:
plain RLS (w = 1) against weighted RLS, with supplied features and with the
paper's temporal feature, each with and without the 5x5 blend, scored by
PSNR against the clean frames of a seeded c2-scene sequence; and the fixed
against the automatic forgetting factor on scenes with and without
appearance edits."""
from __future__ import annotations

import math

import numpy as np

import oracle
import synth

SIGMA_S, SIGMA_R = 1.5, 0.15


def modes(d_features: int):
    """Same modes and priors as bench.ablation_modes (delta in each mode's
    weight units)."""
    return [
        ("rls_features", d_features, dict(wmode=oracle.W_ONE, delta=1.0)),
        ("wrls_features", d_features, dict(wmode=oracle.W_INVVAR, delta=math.exp(-synth.VAR_MU))),
        ("rls_temporal_feature", 4, dict(wmode=oracle.W_PAPER, h_bw=1e3)),
        ("wrls_temporal_feature", 4, dict(wmode=oracle.W_PAPER)),
        ("wrls_features_auto_lambda", d_features, dict(wmode=oracle.W_INVVAR, delta=math.exp(-synth.VAR_MU),
                                                       sigma0=60.0, lam_min=0.5)),
    ]


def psnr(mse: float) -> float:
    return 10.0 * math.log10(1.0 / mse)


def run(width: int, height: int, frames: int, warm: int):
    wl = synth.c2(width=width, height=height, frames=frames)
    src = synth.FrameSource(wl)
    seq = [src.next() for _ in range(frames)]
    res = {"input": {"psnr_db": psnr(float(np.mean([np.mean((f.color.astype(np.float64) - f.clean) ** 2)
                                                     for f in seq[warm:]])))}}
    for name, d, kw in modes(wl.d):
        o = oracle.Oracle(width, height, d, **kw)
        paper = kw["wmode"] == oracle.W_PAPER
        se_t, se_b = [], []
        for t, f in enumerate(seq):
            out = o.step(f.color, None if paper else f.feats,
                         f.var if kw["wmode"] == oracle.W_INVVAR else None, f.motion)
            bl = o.blend(None if paper else f.feats, SIGMA_S, SIGMA_R)
            if t >= warm:
                se_t.append(np.mean((out - f.clean) ** 2))
                se_b.append(np.mean((bl - f.clean) ** 2))
        res[name] = {"psnr_db": psnr(float(np.mean(se_t))), "psnr_blend_db": psnr(float(np.mean(se_b)))}
    return res


# automatic forgetting factor of the ablation: information and lower limit
# (the upper limit is the fixed factor, 0.98)
AUTO_SIGMA0, AUTO_LAM_MIN = 60.0, 0.5


def run_forgetting(scene: str, width: int, height: int, frames: int, warm: int, edit: int):
    """PSNR of weighted RLS with supplied features, fixed lambda = 0.98
    against the automatic factor, over frames warm..end and over edit..end
    (the c3 scene's colour LUT changes at frame 15 and its light at 22; the
    c2 scene has no edit)."""
    wl = (synth.c3 if scene == "c3" else synth.c2)(width=width, height=height, frames=frames)
    src = synth.FrameSource(wl)
    seq = [src.next() for _ in range(frames)]
    delta = math.exp(-synth.VAR_MU)
    res = {}
    for name, kw in (("fixed", {}), ("auto", dict(sigma0=AUTO_SIGMA0, lam_min=AUTO_LAM_MIN))):
        o = oracle.Oracle(width, height, wl.d, lam=0.98, delta=delta, **kw)
        se = [np.mean((o.step(f.color, f.feats, f.var, f.motion) - f.clean) ** 2) for f in seq]
        res[name] = {"psnr_db": psnr(float(np.mean(se[warm:]))),
                     "psnr_after_edit_db": psnr(float(np.mean(se[edit:])))}
    return res


def per_frame_psnr(scene: str, width: int, height: int, frames: int):
    """PSNR against the clean field of every frame of weighted RLS with
    supplied features and fixed lambda = 0.98 (no reset at any frame), and of
    the noisy input, on the c3 scene (colour LUT edit at frame 15, light
    change at 22) or the c2 scene."""
    wl = (synth.c3 if scene == "c3" else synth.c2)(width=width, height=height, frames=frames)
    src = synth.FrameSource(wl)
    o = oracle.Oracle(width, height, wl.d, lam=0.98, delta=math.exp(-synth.VAR_MU))
    out, inp = [], []
    for _ in range(frames):
        f = src.next()
        y = o.step(f.color, f.feats, f.var, f.motion)
        out.append(psnr(float(np.mean((y - f.clean) ** 2))))
        inp.append(psnr(float(np.mean((f.color.astype(np.float64) - f.clean) ** 2))))
    return out, inp
