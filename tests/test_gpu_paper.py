"""Paper mode on the GPU against the FP64 oracle: the temporal feature of
Eq. 12 (3x3 clamp of the reprojected history, blend with the current colour)
as the predictor p = [1, z] and the weight of Eq. 13, d = 4.

Bar: G1/G2/G3 <= 1e-4 as for the other modes (tests/parity.py); the history
z itself within 1e-4 of the oracle's relative to |z| (it is a clamp, a blend
and a bilinear average of binary32 values: a few ulp); bitwise equality for
history export/import.
"""
import numpy as np
import pytest

import synth
from parity import G1_TOL, G2_TOL, G3_TOL, Pair, g1, log, predictor, term_scale, to_dev

pytestmark = pytest.mark.gpu

Z_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2106_08034_amd import wrls
    wrls.lib()
    yield


def _run(wl, frames=None, **kw):
    """wl: a scene workload; its features are generated but not used."""
    src = synth.FrameSource(wl)
    pair = Pair(wl.width, wl.height, 4, in_dtype=wl.in_dtype, weight_mode="paper", **kw)
    n = wl.frames if frames is None else frames
    worst = worst_z = 0.0
    for t in range(n):
        f = src.next()
        log("case paper %s %dx%d frame %d/%d" % (wl.name, wl.width, wl.height, t + 1, n))
        out, ref, e = pair.step(f.color, None, None, f.motion)
        ez = pair.history_error()
        worst, worst_z = max(worst, e), max(worst_z, ez)
        assert e <= G1_TOL, "frame %d: G1 %.3g" % (t, e)
        assert ez <= Z_TOL, "frame %d: history %.3g" % (t, ez)
    e2, e3, eb = pair.state_errors(None)
    assert e2 <= G2_TOL, "G2 %.3g" % e2
    assert e3 <= G3_TOL, "G3 %.3g" % e3
    log("case paper %s: worst G1 %.3g, history %.3g, G2 %.3g, G3 %.3g, beta normwise %.3g"
        % (wl.name, worst, worst_z, e2, e3, eb))
    return pair


def test_paper_c2_pan_ragged_small():
    _run(synth.c2(width=197, height=83, frames=24))


def test_paper_c3_orbit_fp16_with_edits_small():
    _run(synth.c3(width=203, height=117, frames=30))


def test_paper_nearest_and_other_constants():
    _run(synth.c2(width=131, height=37, frames=10), interp="nearest", alpha=0.4, h=0.3,
         eps=1e-2, lam=0.9)


def test_paper_c2_full_size_1080p():
    _run(synth.c2(frames=8))


def test_paper_edge_cases():
    """Non-finite colour (the history is carried, weight 0), black pixels
    (distance 0 / eps), restarts from NaN or off-image motion, borders."""
    rng = np.random.default_rng(11)
    H, W = 12, 67
    pair = Pair(W, H, 4, weight_mode="paper")
    for t in range(6):
        log("case paper edge t=%d" % t)
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        motion = rng.uniform(-1.5, 1.5, size=(2, H, W)).astype(np.float32)
        color[:, 0:3, 0:3] = 0.0                    # a black corner
        color[1, 2 + t % 3, 30] = np.nan
        color[0, 5, 31 + t] = np.inf
        color[:, 7, 40] = -np.inf
        color[2, 8, 0] = 100.0                      # an HDR highlight
        motion[:, 0, 0] = (W - 1, H - 1)
        motion[:, 2, 2] = (np.inf, 0.0)
        motion[:, 4, 4] = (-4.5, 0.0)
        motion[:, 5, 5] = (0.0, np.nan)
        out, ref, e = pair.step(color, None, None, motion)
        assert np.all(np.isfinite(out))
        assert e <= G1_TOL, e
        assert pair.history_error() <= Z_TOL
    e2, e3, _ = pair.state_errors(None)
    assert e2 <= G2_TOL and e3 <= G3_TOL


@pytest.mark.parametrize("level", [1e4, 1e6])
def test_paper_extreme_fireflies_reported(level):
    """Colour far above the scene's range: the colour enters p, so p P p^T
    holds its square (1e8 .. 1e12) and the covariance update P - q p P
    cancels to that factor's reciprocal, below binary32 resolution of P's
    other entries.  The FP32 state then loses accuracy at those pixels
    while the FP64 oracle does not: the error there is reported; the output
    must stay finite and pixels whose motion chains never touch a firefly
    stay within the usual bar."""
    rng = np.random.default_rng(12)
    H, W, T = 16, 64, 5
    pair = Pair(W, H, 4, weight_mode="paper")
    # fireflies sit in columns 5..13; a chain moves at most 1 column left and
    # 2 right per frame (bilinear taps) and the 3x3 clamp window 1 more, so
    # 5 frames reach at most 15 columns further
    far = np.ones((H, W), bool)
    far[:, :32] = False
    worst_all = worst_far = 0.0
    for t in range(T):
        log("case paper firefly %.0e t=%d" % (level, t))
        color = rng.uniform(0, 1.5, size=(3, H, W)).astype(np.float32)
        motion = rng.uniform(-1.0, 1.0, size=(2, H, W)).astype(np.float32)
        color[t % 3, 3 + t, 5 + 2 * t] = level
        out, ref, e = pair.step(color, None, None, motion)
        assert np.all(np.isfinite(out))
        scale = term_scale(pair.ref.get_beta(), predictor(pair.ref.get_history()))
        worst_all = max(worst_all, e)
        worst_far = max(worst_far, g1(out[:, far], ref[:, far], scale[:, far]))
    log("firefly %.0e: worst relative error %.3g overall, %.3g away from fireflies"
        % (level, worst_all, worst_far))
    assert worst_far <= G1_TOL


def test_paper_history_roundtrip_and_import():
    """get_history/set_history are exact; a stream given another stream's
    state and history continues exactly as that stream does."""
    import torch
    from paper_2106_08034_amd import wrls
    wl = synth.c2(width=96, height=40, frames=5)
    src = synth.FrameSource(wl)
    a = wrls.Stream(wl.width, wl.height, 4, weight_mode="paper")
    frames = [src.next() for _ in range(wl.frames)]
    for f in frames[:4]:
        a.step(to_dev(f.color), None, None, to_dev(f.motion))
    P, B = a.get_state()
    z = a.get_history()
    b = wrls.Stream(wl.width, wl.height, 4, weight_mode="paper")
    b.set_state(P, B, frames=4)
    b.set_history(z)
    assert torch.equal(b.get_history(), z)
    f = frames[4]
    oa = a.step(to_dev(f.color), None, None, to_dev(f.motion))
    ob = b.step(to_dev(f.color), None, None, to_dev(f.motion))
    assert torch.equal(oa, ob)
    assert torch.equal(a.get_history(), b.get_history())
    a.close()
    b.close()


def test_paper_reset_clears_history():
    import torch
    from paper_2106_08034_amd import wrls
    wl = synth.c2(width=70, height=20, frames=3)
    src = synth.FrameSource(wl)
    fr = [src.next() for _ in range(3)]
    a = wrls.Stream(wl.width, wl.height, 4, weight_mode="paper")
    for f in fr:
        a.step(to_dev(f.color), None, None, to_dev(f.motion))
    a.reset()
    b = wrls.Stream(wl.width, wl.height, 4, weight_mode="paper")
    for f in fr:
        assert torch.equal(a.step(to_dev(f.color), None, None, to_dev(f.motion)),
                           b.step(to_dev(f.color), None, None, to_dev(f.motion)))
    assert torch.equal(a.get_history(), b.get_history())


def test_batch_rejects_paper_streams():
    from paper_2106_08034_amd import wrls
    s = wrls.Stream(32, 8, 4, weight_mode="paper")
    b = wrls.Batch(2, 4)
    import torch
    c = torch.rand((3, 8, 32), device="cuda")
    with pytest.raises(wrls.WrlsError) as ei:
        b.step([s], [(c, None, None, None)])
    assert ei.value.status == wrls.WRLS_EUNSUPPORTED


def test_paper_every_launch_shape_bitwise():
    """The paper kernel stages a colour halo per tile, so its indexing depends
    on the launch shape: every accepted shape (extremes included: 1-pixel-wide
    tiles, 256 x 1, 16 x 16) must give the default shape's outputs and state
    bitwise, and the default shape matches the oracle."""
    import torch
    from paper_2106_08034_amd import wrls
    wl = synth.c2(width=133, height=41, frames=4)
    src = synth.FrameSource(wl)
    frames = [src.next() for _ in range(wl.frames)]
    pair = Pair(wl.width, wl.height, 4, weight_mode="paper")
    assert pair.gpu.tile == (6, 128, 0)  # paper-mode default: 64 x 2
    outs = []
    for f in frames:
        out, ref, e = pair.step(f.color, None, None, f.motion)
        assert e <= G1_TOL
        outs.append(out)
    P0, B0 = pair.gpu.get_state()
    z0 = pair.gpu.get_history()
    shapes = [(0, 64), (1, 64), (6, 64), (8, 256), (4, 256), (0, 256), (7, 128), (2, 128)]
    for tw, bt in shapes:
        log("case paper shape %dx%d" % (1 << tw, bt >> tw))
        s = wrls.Stream(wl.width, wl.height, 4, weight_mode="paper")
        s.set_tile(tw, bt, 0)
        for t, f in enumerate(frames):
            got = s.step(to_dev(f.color), None, None, to_dev(f.motion))
            assert np.array_equal(got.cpu().numpy(), outs[t]), ((tw, bt), t)
        P, B = s.get_state()
        assert torch.equal(P, P0) and torch.equal(B, B0) and torch.equal(s.get_history(), z0), (tw, bt)
        s.close()
    torch.cuda.synchronize()
