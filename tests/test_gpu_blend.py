"""The 5x5 spatial blend (Sec. 5.3, last paragraph) on the GPU against the
FP64 oracle, after steps run on both sides from identical seeded inputs.

Bar: max |out_gpu - out_ref| / max(|out_ref|, s, tau) <= 1e-4, where s is
the largest term magnitude sum_m |p_i,m beta_k,c,m| among the predictions
the window averages (the scale of the FP32 rounding of those dot products,
as for the step's G1) and tau = 1e-3 RMS(out_ref).  The blend adds 25
weighted terms and one dot product per output (a few ulp on that scale) to
the state's own error, which the step's gates hold at 1e-4.
"""
import numpy as np
import pytest

import synth
from parity import G1_TOL, Pair, blend_scale, g1, log, predictor, to_dev

pytestmark = pytest.mark.gpu

BLEND_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2106_08034_amd import wrls
    wrls.lib()
    yield


def _blend_check(pair, feats, out_t, sigma_s, sigma_r, tag):
    import torch
    paper = pair.paper
    f_dev = None if (paper or pair.d == 1) else to_dev(feats)
    got = pair.gpu.blend(f_dev, out_t, sigma_s, sigma_r)
    torch.cuda.synchronize()
    ref = pair.ref.blend(None if (paper or pair.d == 1) else feats, sigma_s, sigma_r)
    if paper:
        p = predictor(pair.ref.get_history())
    elif pair.d > 1:
        p = np.where(np.isfinite(predictor(feats)), predictor(feats), 0.0)
    else:
        p = np.ones((1,) + ref.shape[1:])
    e = g1(got.cpu().numpy(), ref, blend_scale(pair.ref.get_beta(), p))
    log("blend %s sigma_s=%s sigma_r=%s: error %.3g" % (tag, sigma_s, sigma_r, e))
    assert e <= BLEND_TOL, (tag, sigma_s, sigma_r, e)
    return got


def _run_then_blend(wl, frames, sigmas, weight_mode="invvar", every_frame=False):
    src = synth.FrameSource(wl)
    d = 4 if weight_mode == "paper" else wl.d
    pair = Pair(wl.width, wl.height, d, in_dtype=wl.in_dtype, weight_mode=weight_mode)
    for t in range(frames):
        f = src.next()
        log("case blend %s %s frame %d/%d" % (wl.name, weight_mode, t + 1, frames))
        use_f = weight_mode != "paper"
        out_t = pair.gpu.step(to_dev(f.color), to_dev(f.feats) if use_f else None,
                              to_dev(f.var) if weight_mode == "invvar" else None, to_dev(f.motion))
        ref = pair.ref.step(f.color, f.feats if use_f else None,
                            f.var if weight_mode == "invvar" else None, f.motion)
        if every_frame or t == frames - 1:
            for ss, sr in sigmas:
                _blend_check(pair, f.feats, out_t, ss, sr, "%s t=%d" % (wl.name, t))
    return pair


SIGMAS = [(1.5, 0.15), (2.0, np.inf), (np.inf, np.inf), (1e-3, np.inf), (0.8, 0.02)]


def test_blend_c2_pan_ragged_small():
    _run_then_blend(synth.c2(width=197, height=83, frames=8), 8, SIGMAS, every_frame=True)


def test_blend_c3_orbit_fp16_d10_small():
    _run_then_blend(synth.c3(width=203, height=117, frames=10), 10, SIGMAS[:3])


def test_blend_paper_mode():
    _run_then_blend(synth.c2(width=150, height=45, frames=6), 6, SIGMAS, weight_mode="paper")


def test_blend_c2_full_size_1080p():
    _run_then_blend(synth.c2(frames=4), 4, [(1.5, 0.15)])


def test_blend_c3_full_size_4k():
    # 4K at d = 10 is wide enough that the tiles run in vertical strips;
    # every pixel, strip edges included, is compared.
    _run_then_blend(synth.c3(frames=3), 3, [(1.5, 0.15)])


def test_blend_wide_ragged_rows_in_strips():
    # 3905 px at d = 10: 62 tiles per row (the last one 1 px wide), in strips
    # of 15 tiles and a last strip of 2; two tile rows and a partial third.
    _run_then_blend(synth.c3(width=3905, height=21, frames=3), 3, SIGMAS[:2])


@pytest.mark.parametrize("d", list(range(1, 11)))
def test_blend_every_d(d):
    rng = np.random.default_rng(300 + d)
    H, W = 9, 70
    pair = Pair(W, H, d, lam=0.95)
    for t in range(4):
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        motion = rng.uniform(-1.6, 1.6, size=(2, H, W)).astype(np.float32)
        out, ref, e = pair.step(color, feats, var, motion)
        assert e <= G1_TOL
    import torch
    out_t = torch.from_numpy(out).cuda()
    for ss, sr in [(1.3, 0.2), (np.inf, np.inf)]:
        _blend_check(pair, feats, out_t, ss, sr, "d=%d" % d)


@pytest.mark.parametrize("W,H", [(1, 1), (1, 300), (300, 1), (65, 5), (2, 3)])
def test_blend_degenerate_shapes(W, H):
    rng = np.random.default_rng(W * 13 + H)
    d = 8
    pair = Pair(W, H, d)
    for t in range(3):
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        motion = rng.uniform(-0.8, 0.8, size=(2, H, W)).astype(np.float32)
        out, ref, e = pair.step(color, feats, var, motion)
    import torch
    _blend_check(pair, feats, torch.from_numpy(out).cuda(), 1.5, 0.15, "%dx%d" % (W, H))


def test_blend_nonfinite_features():
    rng = np.random.default_rng(21)
    H, W, d = 12, 67, 8
    pair = Pair(W, H, d)
    for t in range(3):
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        feats[2, 8, 20] = np.nan
        feats[0, 0, 0] = -np.inf
        out, ref, e = pair.step(color, feats, var, None)
    import torch
    got = _blend_check(pair, feats, torch.from_numpy(out).cuda(), 1.5, 0.15, "nonfinite")
    assert torch.isfinite(got).all()


def test_blend_leaves_state_alone_and_rejects_bad_arguments():
    import torch
    from paper_2106_08034_amd import wrls
    W, H, d = 80, 20, 8
    s = wrls.Stream(W, H, d)
    feats = torch.rand((d - 1, H, W), device="cuda")
    color = torch.rand((3, H, W), device="cuda")
    var = torch.full((H, W), 0.05, device="cuda")
    out = torch.empty((3, H, W), device="cuda")
    with pytest.raises(wrls.WrlsError) as ei:       # no state yet
        s.blend(feats, out, 1.5, 0.1)
    assert ei.value.status == wrls.WRLS_EINVAL
    s.step(color, feats, var, None, out=out)
    P0, B0 = s.get_state()
    fin = s.blend(feats, out, 1.5, 0.1)
    P1, B1 = s.get_state()
    assert torch.equal(P0, P1) and torch.equal(B0, B1)
    for ss, sr in [(0.0, 0.1), (1.0, -1.0), (float("nan"), 1.0), (1e-30, 1.0)]:
        with pytest.raises(wrls.WrlsError) as ei:
            s.blend(feats, out, ss, sr)
        assert ei.value.status == wrls.WRLS_EINVAL
    with pytest.raises(wrls.WrlsError):            # output aliasing the guide
        s.blend(feats, out, 1.5, 0.1, out=out)
    # misaligned arrays are rejected on the host, before any launch
    L = wrls.lib()
    odd = fin.data_ptr() + 2
    assert L.wrls_blend(s.handle, feats.data_ptr(), out.data_ptr(), 1.5, 0.1, odd) == wrls.WRLS_EINVAL
    assert L.wrls_step(s.handle, color.data_ptr(), feats.data_ptr() + 1, var.data_ptr(), None,
                       out.data_ptr()) == wrls.WRLS_EINVAL
    assert L.wrls_step(s.handle, color.data_ptr(), feats.data_ptr(), var.data_ptr(), None,
                       color.data_ptr()) == wrls.WRLS_EINVAL
    assert s.frames == 1
    assert torch.isfinite(fin).all()
    s.close()
