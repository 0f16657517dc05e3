"""Every kernel access stays inside its array.  libwrls_checked.so is the
same source built with its access checks on (each reprojection tap, each
16-byte state access or store and each LDS index is tested before use; a
failing access is skipped and its site flagged).  It runs edge cases that
push the addressing to its limits: degenerate and ragged shapes, every d,
both input types, bilinear and nearest reprojection, motion that lands
exactly on the image border, just outside it, far outside it, or is not
finite; the full-size scenes (the spatial blend in strip order at 4K), paper
mode, the traffic probe, batched steps on both grids and the allocation-free
batched step.
Bar: no site flagged, and every output and final state bitwise equal to the
shipped library's on the same inputs."""
import os

import numpy as np
import pytest

import synth
from parity import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def libs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2106_08034_amd import wrls
    shipped = wrls.lib()
    saved = wrls.LIB_PATH
    wrls._lib = None
    wrls.LIB_PATH = os.path.join(os.path.dirname(saved), "libwrls_checked.so")
    try:
        checked = wrls.lib()
    finally:
        wrls.LIB_PATH = saved
        wrls._lib = shipped
    assert checked.wrls_checked_build() == 1 and shipped.wrls_checked_build() == 0
    yield {"shipped": shipped, "checked": checked}
    wrls._lib = shipped


def test_checked_flags_reach_the_host(libs):
    """The reporting path itself: flags raised from a kernel are read back
    once per site and cleared by the read."""
    import torch
    from paper_2106_08034_amd import wrls
    wrls._lib = libs["checked"]
    try:
        assert wrls.wrls_checked_failures() == 0
        for mask in (1, 1 << 3, (1 << len(wrls.CHECK_SITES)) - 1):
            wrls.wrls_checked_raise(mask)
            torch.cuda.synchronize()
            assert wrls.wrls_checked_failures() == mask, mask
            assert wrls.wrls_checked_failures() == 0
    finally:
        wrls._lib = libs["shipped"]


def _edge_motion(rng, W, H):
    """Per pixel, a horizontal and a vertical displacement drawn from the
    cases that decide the gather's taps: exactly on the first or last
    column/row, a hair inside or outside, far outside, sub-pixel, negative
    fractions and non-finite values."""
    x = np.arange(W, dtype=np.float64)[None, :].repeat(H, 0)
    y = np.arange(H, dtype=np.float64)[:, None].repeat(W, 1)

    def pick(pos, n):
        cases = np.stack([-pos, (n - 1) - pos, -pos - 1e-3, (n - 1) - pos + 1e-3, -pos + 1e-6,
                          (n - 1) - pos - 1e-6, np.full_like(pos, 0.5), np.full_like(pos, -0.25),
                          np.full_like(pos, -1e-8), np.full_like(pos, 3.7e9), np.full_like(pos, -2.5e9),
                          np.full_like(pos, np.nan), np.full_like(pos, np.inf), np.full_like(pos, -np.inf),
                          np.zeros_like(pos)])
        k = rng.integers(0, cases.shape[0], size=pos.shape)
        return np.take_along_axis(cases, k[None], 0)[0].astype(np.float32)

    return np.stack([pick(x, W), pick(y, H)])


def _frames(seed, W, H, d, f16, T):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(T):
        c = rng.normal(0.5, 0.3, (3, H, W))
        fe = rng.normal(0.0, 1.0, (d - 1, H, W)) if d > 1 else np.zeros((0, H, W))
        v = rng.lognormal(-3.0, 1.0, (H, W)).astype(np.float32)
        m = _edge_motion(rng, W, H)
        dt = np.float16 if f16 else np.float32
        out.append((c.astype(dt), fe.astype(dt), v, m))
    return out


def _run(wrls, L, W, H, d, f16, frames, mode, interp, tile=None):
    """Steps, probes and blends one stream with library L; returns the
    outputs and the final state (host copies)."""
    import torch
    wrls._lib = L
    paper = mode == "paper"
    s = wrls.Stream(W, H, d, in_dtype="f16" if f16 else "f32", weight_mode=mode,
                    interp=interp)
    if tile is not None:
        s.set_tile(*tile)
    res = []
    for t, f in enumerate(frames):
        c, fe, v, m = (to_dev(a) for a in f)
        fe = None if (paper or d == 1) else fe
        v = None if paper else v
        if t == 1:
            s.traffic_probe(c, fe, v, m)
        out = s.step(c, fe, v, m)
        res.append(out.cpu())
        res.append(s.blend(fe, out, 1.5, 0.15).cpu())
    P, B = s.get_state()
    res += [P.cpu(), B.cpu()]
    if paper:
        res.append(s.get_history().cpu())
    s.close()
    torch.cuda.synchronize()
    return res


def _compare(libs, tag, fn):
    import torch
    from paper_2106_08034_amd import wrls
    a = fn(wrls, libs["shipped"])
    b = fn(wrls, libs["checked"])
    wrls._lib = libs["checked"]
    flags = wrls.wrls_checked_failures()
    wrls._lib = libs["shipped"]
    bad = [wrls.CHECK_SITES[i] for i in range(len(wrls.CHECK_SITES)) if flags >> i & 1]
    log("checked %s: %d arrays, failed sites %s" % (tag, len(a), bad or "none"))
    assert not bad, (tag, bad)
    for i, (x, y) in enumerate(zip(a, b)):
        assert torch.equal(x, y) or (torch.isnan(x).equal(torch.isnan(y)) and
                                     torch.equal(torch.nan_to_num(x), torch.nan_to_num(y))), (tag, i)


SHAPES = [(1, 1), (1, 300), (300, 1), (65, 5), (2, 3), (197, 83), (256, 17)]


@pytest.mark.parametrize("d", [1, 4, 8, 10])
@pytest.mark.parametrize("f16", [False, True])
def test_checked_steps_blend_probe(libs, d, f16):
    for k, (W, H) in enumerate(SHAPES):
        frames = _frames(1000 * d + 10 * k + f16, W, H, d, f16, 3)
        for interp in ("bilinear", "nearest"):
            _compare(libs, "d=%d f16=%s %dx%d %s" % (d, f16, W, H, interp),
                     lambda wrls, L: _run(wrls, L, W, H, d, f16, frames, "invvar", interp))


def test_checked_paper_mode_and_tiles(libs):
    for k, (W, H) in enumerate(SHAPES):
        frames = _frames(77 + k, W, H, 4, False, 3)
        for tile in (None, (7, 128, 0), (5, 128, 0), (6, 256, 3)):
            _compare(libs, "paper %dx%d tile %s" % (W, H, tile),
                     lambda wrls, L: _run(wrls, L, W, H, 4, False, frames, "paper", "bilinear",
                                          tile))


@pytest.mark.parametrize("scene", ["c3", "c2", "c2_paper"])
def test_checked_full_size_scenes(libs, scene):
    # 4K d = 10 FP16 (the blend in strips), 1080p d = 8 FP32 and 1080p paper
    # mode, with the scenes' own motion fields and disocclusions
    wl = synth.c3(frames=3) if scene == "c3" else synth.c2(frames=3)
    src = synth.FrameSource(wl)
    frames = []
    for _ in range(3):
        f = src.next()
        frames.append((f.color, f.feats, f.var, f.motion))
    paper = scene == "c2_paper"
    _compare(libs, "%s %dx%d" % (scene, wl.width, wl.height),
             lambda wrls, L: _run(wrls, L, wl.width, wl.height, 4 if paper else wl.d,
                                  wl.in_dtype == "f16", frames, "paper" if paper else "invvar",
                                  "bilinear"))


def _batch_run(wrls, L, wls, frames, blocks_per_cu, noalloc):
    import torch
    wrls._lib = L
    streams = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16") for wl in wls]
    outs = [torch.empty((3, wl.height, wl.width), device="cuda") for wl in wls]
    b = None if noalloc else wrls.Batch(len(wls), 8, "f16", use_graph=blocks_per_cu == 0)
    if b is not None:
        b.set_tile(7, 128, blocks_per_cu)
    res = []
    for t in range(len(frames[0])):
        fr = [tuple(to_dev(a) for a in frames[i][t]) for i in range(len(wls))]
        if noalloc:
            wrls.wrls_batch_step_noalloc([s.handle for s in streams], [f + (o,) for f, o in zip(fr, outs)])
        else:
            b.step(streams, fr, outs)
        torch.cuda.synchronize()
        res += [o.cpu() for o in outs]
    for s in streams:
        P, B = s.get_state()
        res += [P.cpu(), B.cpu()]
        s.close()
    if b is not None:
        b.close()
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("blocks_per_cu,noalloc", [(0, False), (1, False), (-1, False), (0, True)])
def test_checked_batched_steps(libs, blocks_per_cu, noalloc):
    sizes = [(197, 83), (1, 1), (65, 5), (320, 240), (2, 3), (300, 1)]
    frames = [_frames(500 + i, W, H, 8, True, 3) for i, (W, H) in enumerate(sizes)]

    class WL:
        def __init__(self, W, H):
            self.width, self.height = W, H

    wls = [WL(W, H) for W, H in sizes]
    _compare(libs, "batch blocks_per_cu=%d noalloc=%s" % (blocks_per_cu, noalloc),
             lambda wrls, L: _batch_run(wrls, L, wls, frames, blocks_per_cu, noalloc))
