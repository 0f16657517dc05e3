"""GPU (libwrls, gfx950) against the FP64 oracle on identical seeded inputs.

Bar: G1/G2/G3 <= 1e-4 (see tests/parity.py) for floating point; bitwise
equality where the method is exact (reset == fresh stream, state
export/import, zero-weight ageing of a constant state).
"""
import numpy as np
import pytest

import synth
from parity import (G1_TOL, G2_TOL, G3_TOL, S_RMS_BOUND, Pair, g1, log, predictor, term_scale,
                    to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2106_08034_amd import wrls
    wrls.lib()
    yield


def _run(wl, frames=None, check_state=True, **kw):
    src = synth.FrameSource(wl)
    pair = Pair(wl.width, wl.height, wl.d, in_dtype=wl.in_dtype, **kw)
    n = wl.frames if frames is None else frames
    worst = 0.0
    for t in range(n):
        f = src.next()
        log("case %s frame %d/%d" % (wl.name, t + 1, n))
        out, ref, e = pair.step(f.color, f.feats, f.var, f.motion)
        worst = max(worst, e)
        assert e <= G1_TOL, "frame %d: G1 %.3g" % (t, e)
    e2 = e3 = eb = None
    if check_state:
        e2, e3, eb = pair.state_errors(f.feats)
        assert e2 <= G2_TOL, "G2 %.3g" % e2
        assert e3 <= G3_TOL, "G3 %.3g" % e3
    log("case %s: worst G1 %.3g, G2 %s, G3 %s, beta normwise (reported) %s; %s"
        % (wl.name, worst, e2, e3, eb, pair.relaxation()))
    assert pair.s_rms_max <= S_RMS_BOUND, pair.relaxation()
    return worst


def test_c1_static_64x64_all_frames():
    _run(synth.c1())


def test_c2_pan_ragged_small():
    # several 64x4 tiles plus a ragged tail in both directions
    _run(synth.c2(width=197, height=83, frames=24))


def test_c3_orbit_fp16_d10_with_edits_small():
    wl = synth.c3(width=203, height=117, frames=30)
    _run(wl)


def test_c3_fp16_error_against_unrounded_inputs_reported():
    """FP16 inputs: the error of the GPU run against an oracle fed the
    unrounded FP32 inputs is reported.  It measures the binary16 rounding of
    colour and features (relative 2^-11 per value), not the kernel, and stays
    within a small multiple of that rounding on the term scale."""
    import oracle
    from paper_2106_08034_amd import wrls
    wl = synth.c3(width=96, height=64, frames=12)
    src = synth.FrameSource(wl)
    g = wrls.Stream(wl.width, wl.height, wl.d, in_dtype="f16")
    o32 = oracle.Oracle(wl.width, wl.height, wl.d)
    worst = 0.0
    for t in range(wl.frames):
        f = src.next(keep_unrounded=True)
        out = g.step(to_dev(f.color), to_dev(f.feats), to_dev(f.var), to_dev(f.motion)).cpu().numpy()
        ref = o32.step(f.color_f32, f.feats_f32, f.var, f.motion)
        scale = term_scale(o32.get_beta(), predictor(f.feats_f32))
        worst = max(worst, g1(out, ref, scale))
    log("FP16 inputs vs unrounded-FP32 oracle: max rel error (term scale) %.3g" % worst)
    assert worst < 50 * 2.0 ** -11


@pytest.mark.parametrize("d", list(range(1, 11)))
@pytest.mark.parametrize("interp", ["bilinear", "nearest"])
@pytest.mark.parametrize("weight_mode", ["invvar", "one"])
def test_modes_and_every_d(d, interp, weight_mode):
    rng = np.random.default_rng(100 + d)
    H, W, T = 9, 70, 6
    pair = Pair(W, H, d, lam=0.95, delta=0.5, interp=interp, weight_mode=weight_mode)
    log("case d=%d %s %s" % (d, interp, weight_mode))
    for t in range(T):
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        motion = rng.uniform(-1.6, 1.6, size=(2, H, W)).astype(np.float32)
        motion[:, rng.random((H, W)) < 0.05] = np.nan
        out, ref, e = pair.step(color, feats, var if weight_mode == "invvar" else None, motion)
        assert e <= G1_TOL, e
    e2, e3, _ = pair.state_errors(feats)
    assert e2 <= G2_TOL and e3 <= G3_TOL


def test_edge_cases_nonfinite_inputs_and_borders():
    rng = np.random.default_rng(7)
    H, W, d = 12, 67, 8
    pair = Pair(W, H, d)
    for t in range(5):
        log("case edge t=%d" % t)
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        motion = rng.uniform(-1, 1, size=(2, H, W)).astype(np.float32)
        color[1, 2, 3] = np.nan
        color[0, 4, 5] = np.inf
        var[3, 7] = np.inf
        var[5, 9] = -1.0
        var[6, 11] = 0.0          # floored
        var[7, 13] = np.nan
        feats[2, 8, 20] = np.nan
        feats[0, 9, 21] = -np.inf
        motion[:, 0, 0] = (W - 1, H - 1)            # lands exactly on the last pixel
        motion[:, 1, 0] = (W - 0.5, 0.0)            # lands between the last column and W
        motion[:, 2, 2] = (np.inf, 0.0)
        motion[:, 3, 3] = (0.0, -np.inf)
        motion[:, 4, 4] = (-4.5, 0.0)               # left of the image
        motion[:, 5, 5] = (0.0, np.nan)
        out, ref, e = pair.step(color, feats, var, motion)
        assert np.all(np.isfinite(out))
        assert e <= G1_TOL, e
    e2, e3, _ = pair.state_errors(feats)
    assert e2 <= G2_TOL and e3 <= G3_TOL


@pytest.mark.parametrize("W,H", [(1, 1), (1, 300), (300, 1), (65, 5), (16384, 2)])
def test_degenerate_and_maximum_shapes(W, H):
    rng = np.random.default_rng(W * 7 + H)
    d = 8
    pair = Pair(W, H, d)
    log("case shape %dx%d" % (W, H))
    for t in range(4):
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        motion = rng.uniform(-1.2, 1.2, size=(2, H, W)).astype(np.float32)
        out, ref, e = pair.step(color, feats, var, motion)
        assert e <= G1_TOL, e


def test_exact_source_position_at_large_coordinates():
    """pi(v_j) = j + v_j is taken without rounding at any x: on a
    16384-pixel-wide image (binary32 spacing 2^-10 near the right edge) with
    sub-pixel motions of both signs, the GPU matches the oracle's exact
    taps and weights; a source one binary32 step of the motion past the last
    column (which x + v in binary32 would round onto it) restarts on both
    sides, and one exactly on it does not."""
    rng = np.random.default_rng(31)
    W, H, d = 16384, 3, 4
    pair = Pair(W, H, d)
    up = np.nextafter(np.float32(2.0), np.float32(3.0))
    for t in range(4):
        log("case large coordinates t=%d" % t)
        feats = rng.uniform(0, 1, size=(d - 1, H, W)).astype(np.float32)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        var = np.exp(-3 + rng.standard_normal((H, W))).astype(np.float32)
        motion = np.zeros((2, H, W), np.float32)
        motion[0] = rng.choice(np.array([0.3, -0.7, 1.17, -2.61, 0.013, -1e-9], np.float32), size=(H, W))
        motion[1] = rng.choice(np.array([0.25, -0.4, 0.0], np.float32), size=(H, W))
        motion[1, 0] = np.abs(motion[1, 0])
        motion[1, H - 1] = -np.abs(motion[1, H - 1])
        motion[0, :, W - 3] = (2.0, up, 2.0)
        motion[1, :, W - 3] = 0.0
        out, ref, e = pair.step(color, feats, var, motion)
        assert e <= G1_TOL, e
    e2, e3, _ = pair.state_errors(feats)
    assert e2 <= G2_TOL and e3 <= G3_TOL


def test_reset_equals_fresh_and_state_roundtrip_bitwise():
    import torch
    from paper_2106_08034_amd import wrls
    wl = synth.c2(width=130, height=40, frames=8)
    fr = [(to_dev(f.color), to_dev(f.feats), to_dev(f.var), to_dev(f.motion))
          for f in synth.frames(wl)]
    a = wrls.Stream(wl.width, wl.height, wl.d)
    for f in fr[:4]:
        a.step(*f)
    P, B = a.get_state()
    P, B = P.clone(), B.clone()
    # export -> import into a new stream -> continue: bitwise equal
    b = wrls.Stream(wl.width, wl.height, wl.d)
    b.set_state(P, B, frames=4)
    assert b.frames == 4
    for f in fr[4:]:
        oa = a.step(*f).clone()
        ob = b.step(*f).clone()
        assert torch.equal(oa, ob)
    # reset == fresh stream
    a.reset()
    c = wrls.Stream(wl.width, wl.height, wl.d)
    for f in fr[:3]:
        assert torch.equal(a.step(*f).clone(), c.step(*f).clone())
    torch.cuda.synchronize()


def test_zero_weight_ages_constant_state_exactly():
    """A spatially constant state is reproduced exactly by the bilinear
    gather (nested lerps), and weight 0 only divides P by lambda."""
    import torch
    from paper_2106_08034_amd import wrls
    H, W, d = 16, 80, 4
    s = wrls.Stream(W, H, d, lam=0.5, delta=1.0)
    npk = d * (d + 1) // 2
    P = torch.arange(1, npk + 1, dtype=torch.float32, device="cuda")[:, None, None].expand(npk, H, W).contiguous()
    B = torch.linspace(-1, 1, 3 * d, device="cuda").reshape(3, d, 1, 1).expand(3, d, H, W).contiguous()
    s.set_state(P, B, frames=1)
    rng = np.random.default_rng(3)
    mot = np.stack([rng.uniform(0, W - 1, (H, W)) - np.arange(W)[None, :],
                    rng.uniform(0, H - 1, (H, W)) - np.arange(H)[:, None]]).astype(np.float32)
    feats = torch.rand((d - 1, H, W), device="cuda")
    color = torch.rand((3, H, W), device="cuda")
    var = torch.full((H, W), float("inf"), device="cuda")
    s.step(color, feats, var, to_dev(mot))
    P2, B2 = s.get_state()
    assert torch.equal(P2, P * 2.0)
    assert torch.equal(B2, B)


def test_c2_full_size_1080p_all_60_frames():
    """The benchmark workload itself, in the benchmark's launch
    configuration: every pixel of every frame against the oracle."""
    _run(synth.c2())


def test_c3_full_size_4k_all_30_frames():
    """The full 4K d = 10 FP16 recipe, every pixel of all 30 frames, through
    the colour-LUT edit (frame 15) and the light change (frame 22)."""
    _run(synth.c3())


def _max_square_side(d):
    from paper_2106_08034_amd import wrls
    side = 16384
    while wrls.wrls_params_validate(wrls.wrls_params_default(side, side, d)) != 0:
        side -= 16
    return side


def test_maximum_size_d10_sampled_windows():
    """The largest square image a d = 10 stream accepts (state copy just
    below 4 GiB), FP16 inputs, a sub-pixel pan.  A pixel's model depends only
    on the pixels its motion chain visits, so crops whose chains stay inside
    them are run through small oracles and compared pixel by pixel.  The
    source position j + v is exact on both sides, so a crop sees the taps
    and bilinear weights of the full image at any x (here up to ~3550,
    where a binary32 sum x + v would be off by up to 1.2e-4 px)."""
    import oracle
    import torch
    from paper_2106_08034_amd import wrls
    side = _max_square_side(10)
    T, d, vx = 3, 10, 2.3
    wl = synth.c3(width=side, height=side, frames=T, motion="pan", pan=(vx, 0.0), lut_frame=None,
                  light_frame=None)
    log("case max size %dx%d d=10 (%.1f Mpixel)" % (side, side, side * side / 1e6))
    g = wrls.Stream(side, side, d, in_dtype="f16")
    src = synth.FrameSource(wl)
    wins = [(0, 0), (side - 48, side - 6), (side // 2 + 5, side // 3), (side - 8 - int(vx * T) - 3, 7)]
    w, h = 40, 6
    crops = [(x0, y0, min(side, x0 + w + int(vx * T) + 3), y0 + h) for (x0, y0) in wins]
    oracles = [oracle.Oracle(c[2] - c[0], c[3] - c[1], d) for c in crops]
    for t in range(T):
        f = src.next()
        out = g.step(to_dev(f.color), to_dev(f.feats), to_dev(f.var), to_dev(f.motion))
        torch.cuda.synchronize()
        for (x0, y0, x1, y1), o in zip(crops, oracles):
            ref = o.step(f.color[:, y0:y1, x0:x1], f.feats[:, y0:y1, x0:x1], f.var[y0:y1, x0:x1],
                         f.motion[:, y0:y1, x0:x1])
            scale = term_scale(o.get_beta(), predictor(f.feats[:, y0:y1, x0:x1]))
            n_ok = min(w, (x1 - x0) - int(vx * (t + 1)) - 2)  # columns whose chains stay inside
            got = out[:, y0:y1, x0:x0 + n_ok].cpu().numpy()
            e = g1(got, ref[:, :, :n_ok], scale[:, :, :n_ok])
            assert e <= G1_TOL, (t, x0, y0, e)
    g.close()
    torch.cuda.synchronize()


def test_every_launch_shape_bitwise_and_default_shapes():
    """Results do not depend on the launch shape: every accepted tile shape
    and strip width gives the default shape's outputs and state bitwise.  The
    default is 256 x 1 when 256 divides the width, else 128 x 1."""
    import torch
    from paper_2106_08034_amd import wrls
    assert wrls.Stream(512, 8, 8).tile == (8, 256, 0)
    assert wrls.Stream(1920, 8, 8).tile == (7, 128, 0)
    wl = synth.c2(width=197, height=45, frames=4)
    frames = [tuple(to_dev(x) for x in (f.color, f.feats, f.var, f.motion)) for f in synth.frames(wl)]
    ref = wrls.Stream(wl.width, wl.height, wl.d)
    outs = [ref.step(*f).clone() for f in frames]
    P0, B0 = ref.get_state()
    shapes = [(0, 64, 0), (1, 64, 3), (6, 64, 0), (8, 256, 0), (8, 256, 1), (4, 256, 2), (0, 256, 0),
              (7, 128, 2), (2, 128, 5)]
    for tw, bt, sw in shapes:
        log("case step shape %dx%d strip %d" % (1 << tw, bt >> tw, sw))
        s = wrls.Stream(wl.width, wl.height, wl.d)
        s.set_tile(tw, bt, sw)
        for t, f in enumerate(frames):
            assert torch.equal(s.step(*f), outs[t]), ((tw, bt, sw), t)
        P, B = s.get_state()
        assert torch.equal(P, P0) and torch.equal(B, B0), (tw, bt, sw)
        s.close()
    torch.cuda.synchronize()


def test_device_copy_bitwise():
    """The library's copy kernel (the benchmark's bandwidth reference) copies
    every byte, including a tail that is not a whole workgroup, and leaves
    the bytes past the end untouched."""
    import torch
    from paper_2106_08034_amd import wrls
    g = torch.Generator(device="cuda").manual_seed(5)
    for n in (4, 1000, 1 << 20, (1 << 22) + 68):
        src = torch.randn(n, device="cuda", generator=g)
        dst = torch.full((n + 64,), 7.0, device="cuda")
        wrls.wrls_device_copy(dst, src)
        assert torch.equal(dst[:n], src) and torch.all(dst[n:] == 7.0), n
    with pytest.raises(wrls.WrlsError):
        wrls.wrls_device_copy(dst, src[1:5])  # misaligned source
    torch.cuda.synchronize()


@pytest.mark.parametrize("case", ["c2_d8_f32", "c3_d10_f16", "paper_d4"])
def test_traffic_probe_leaves_the_stream_alone(case):
    """wrls_traffic_probe (the step's loads and stores without reprojection
    or arithmetic, the benchmark's reference) run between two steps changes
    nothing: the later steps' outputs and the final state are bitwise those
    of a stream that never ran it.  Its output channels 1 and 2 are the
    colour it read (widened to FP32)."""
    import torch
    from paper_2106_08034_amd import wrls
    wl = synth.c3(width=203, height=77, frames=4) if case == "c3_d10_f16" else \
        synth.c2(width=197, height=83, frames=4)
    paper = case == "paper_d4"
    d = 4 if paper else wl.d
    mode = "paper" if paper else "invvar"
    src = synth.FrameSource(wl)
    frames = []
    for _ in range(4):
        f = src.next()
        frames.append((to_dev(f.color), None if paper else to_dev(f.feats),
                       None if paper else to_dev(f.var), to_dev(f.motion)))
    log("case traffic probe %s" % case)
    a = wrls.Stream(wl.width, wl.height, d, in_dtype=wl.in_dtype, weight_mode=mode)
    b = wrls.Stream(wl.width, wl.height, d, in_dtype=wl.in_dtype, weight_mode=mode)
    for t, f in enumerate(frames):
        if t == 2:
            po = a.traffic_probe(*f)
            torch.cuda.synchronize()
            assert torch.equal(po[1:], f[0][1:].float()), case
            assert a.frames == 2, a.frames
        oa, ob = a.step(*f), b.step(*f)
        assert torch.equal(oa, ob), (case, t)
    Pa, Ba = a.get_state()
    Pb, Bb = b.get_state()
    assert torch.equal(Pa, Pb) and torch.equal(Ba, Bb), case
    if paper:
        assert torch.equal(a.get_history(), b.get_history()), case
    with pytest.raises(wrls.WrlsError):
        wrls.wrls_traffic_probe(a.handle, None, frames[0][1], frames[0][2], frames[0][3], po)  # no colour
    a.close()
    b.close()
    torch.cuda.synchronize()
