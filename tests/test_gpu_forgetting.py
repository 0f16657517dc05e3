"""The automatic forgetting factor (Fortescue, Kershenbaum and Ydstie's rule;
the paper leaves lambda's selection to future work, Sec. 7.6) on the GPU
against the FP64 oracle, at the bar of the fixed factor (G1-G3 <= 1e-4);
its constant limits give the fixed-factor kernel's bits; batched steps give
the per-frame kernel's bits."""
import numpy as np
import pytest

import synth
from parity import G1_TOL, G2_TOL, G3_TOL, S_RMS_BOUND, Pair, log, to_dev

pytestmark = pytest.mark.gpu

SIGMA0, LAM_MIN = 60.0, 0.5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2106_08034_amd import wrls
    wrls.lib()
    yield


def test_c3_recipe_through_the_appearance_edits():
    """The 4K recipe's orbit, FP16 d = 10, on a ragged crop for all 30 frames:
    the LUT edit at frame 15 and the light change at 22 drive lambda down to
    its lower limit at many pixels."""
    wl = synth.c3(width=203, height=117, frames=30)
    src = synth.FrameSource(wl)
    pair = Pair(wl.width, wl.height, wl.d, in_dtype=wl.in_dtype, sigma0=SIGMA0, lam_min=LAM_MIN)
    worst = 0.0
    for t in range(wl.frames):
        f = src.next()
        log("case auto-lambda c3 crop frame %d" % t)
        out, ref, e = pair.step(f.color, f.feats, f.var, f.motion)
        worst = max(worst, e)
        assert e <= G1_TOL, (t, e)
    e2, e3, eb = pair.state_errors(f.feats)
    log("auto lambda c3 crop: worst G1 %.3g, G2 %.3g, G3 %.3g (beta normwise %.3g); %s"
        % (worst, e2, e3, eb, pair.relaxation()))
    assert e2 <= G2_TOL and e3 <= G3_TOL
    assert pair.s_rms_max <= S_RMS_BOUND


@pytest.mark.parametrize("d", [1, 2, 4, 8, 10])
@pytest.mark.parametrize("weight_mode", ["invvar", "one"])
def test_every_mode_random_inputs(d, weight_mode):
    """Random inputs with outliers, disocclusions and a jump in colour at
    frame 4, which drives lambda to its lower limit at many pixels."""
    rng = np.random.default_rng(200 + d)
    H, W, T = 9, 70, 7
    sigma0 = SIGMA0 if weight_mode == "invvar" else 0.5
    pair = Pair(W, H, d, lam=0.97, delta=0.5, weight_mode=weight_mode, sigma0=sigma0, lam_min=0.4)
    log("case auto-lambda d=%d %s" % (d, weight_mode))
    for t in range(T):
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = (rng.uniform(0, 1.5, size=(3, H, W)) + (3.0 if t >= 4 else 0.0)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        var[rng.random((H, W)) < 0.03] = np.inf
        motion = rng.uniform(-1.6, 1.6, size=(2, H, W)).astype(np.float32)
        motion[:, rng.random((H, W)) < 0.05] = np.nan
        out, ref, e = pair.step(color, feats, var if weight_mode == "invvar" else None, motion)
        assert np.all(np.isfinite(out))
        assert e <= G1_TOL, (t, e)
    e2, e3, _ = pair.state_errors(feats)
    assert e2 <= G2_TOL and e3 <= G3_TOL


def test_paper_mode_with_automatic_lambda():
    wl = synth.c2(width=150, height=70, frames=10)
    src = synth.FrameSource(wl)
    pair = Pair(wl.width, wl.height, 4, weight_mode="paper", sigma0=2.0, lam_min=LAM_MIN)
    for t in range(wl.frames):
        f = src.next()
        out, ref, e = pair.step(f.color, None, None, f.motion)
        assert e <= G1_TOL, (t, e)
    e2, e3, _ = pair.state_errors(None)
    assert e2 <= G2_TOL and e3 <= G3_TOL


@pytest.mark.parametrize("limit", ["sigma0_inf", "lam_min_eq_lambda"])
def test_constant_limits_are_the_fixed_factor_bitwise(limit):
    """sigma0 = +inf leaves the root at 1, clamped to lambda; lambda_min =
    lambda pins it: either way the outputs and state are the fixed-factor
    stream's bits."""
    import torch
    from paper_2106_08034_amd import wrls
    wl = synth.c2(width=197, height=45, frames=5)
    frames = [tuple(to_dev(x) for x in (f.color, f.feats, f.var, f.motion)) for f in synth.frames(wl)]
    fixed = wrls.Stream(wl.width, wl.height, wl.d, lam=0.98)
    kw = dict(sigma0=float("inf"), lam_min=0.5) if limit == "sigma0_inf" else dict(sigma0=SIGMA0, lam_min=0.98)
    auto = wrls.Stream(wl.width, wl.height, wl.d, lam=0.98, **kw)
    for f in frames:
        assert torch.equal(fixed.step(*f), auto.step(*f))
    P0, B0 = fixed.get_state()
    P1, B1 = auto.get_state()
    assert torch.equal(P0, P1) and torch.equal(B0, B1)
    torch.cuda.synchronize()


def test_batched_equals_alone_bitwise():
    import torch
    from paper_2106_08034_amd import wrls
    wls = synth.c4_streams(frames=4, scale=0.1)[:4]
    cs = torch.cuda.current_stream().cuda_stream
    kw = dict(in_dtype="f16", sigma0=SIGMA0, lam_min=LAM_MIN)
    alone = [wrls.Stream(wl.width, wl.height, 8, **kw) for wl in wls]
    mixed = [wrls.Stream(wl.width, wl.height, 8, hip_stream=cs, **kw) for wl in wls]
    b = wrls.Batch(len(wls), 8, "f16", hip_stream=cs)
    srcs = [synth.FrameSource(wl) for wl in wls]
    for t in range(4):
        fr = [tuple(to_dev(x) for x in (f.color, f.feats, f.var, f.motion)) for f in (s.next() for s in srcs)]
        outs = b.step(mixed, fr)
        for s, f, o in zip(alone, fr, outs):
            assert torch.equal(s.step(*f), o), t
    b.close()
    torch.cuda.synchronize()
