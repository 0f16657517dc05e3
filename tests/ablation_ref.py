"""The ablation of Sec. 5.3's design choices computed with the FP64 oracle:
plain RLS (w = 1) against weighted RLS, with supplied features and with the
paper's temporal feature, each with and without the 5x5 blend, scored by
PSNR against the clean frames of a seeded c2-scene sequence."""
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
