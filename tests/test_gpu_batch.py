"""Batched persistent steps on the GPU: every stream's result is bitwise the
same alone (wrls_step) and in the mix (wrls_batch_step, graph replay or plain
launch), whatever else is in the batch; and matches the FP64 oracle."""
import numpy as np
import pytest

import synth
from parity import G1_TOL, g1, log, predictor, term_scale, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    yield


def _mix(scale, frames, n=None):
    wls = synth.c4_streams(frames=frames, scale=scale)
    return wls[:n] if n else wls


def _frames(wl, n):
    src = synth.FrameSource(wl)
    return [src.next() for _ in range(n)]


def _dev(f):
    return (to_dev(f.color), to_dev(f.feats), to_dev(f.var), to_dev(f.motion))


def _tiles(wls, shape):
    tw, bt = 1 << shape[0], shape[1]
    th = bt // tw
    return sum(((wl.width + tw - 1) // tw) * ((wl.height + th - 1) // th) for wl in wls)


@pytest.mark.parametrize("blocks_per_cu", [0, 1, -1])
def test_batch_equals_alone_bitwise_and_matches_oracle(blocks_per_cu):
    """blocks_per_cu 0: one workgroup per tile; 1 and -1: a fixed persistent
    grid (one workgroup per CU, or as many as are resident) whose workgroups
    loop over the tiles, advancing through the frame table as they go."""
    import oracle
    import torch
    from paper_2106_08034_amd import wrls
    T = 6
    wls = _mix(0.1, T, n=6)
    host = [_frames(wl, T) for wl in wls]
    dev = [[_dev(f) for f in fr] for fr in host]
    alone = [wrls.Stream(wl.width, wl.height, wl.d, in_dtype="f16") for wl in wls]
    b_graph = wrls.Batch(len(wls), 8, "f16")
    cs = b_graph.hip_stream
    mixed = [wrls.Stream(wl.width, wl.height, wl.d, in_dtype="f16", hip_stream=cs) for wl in wls]
    b_plain = wrls.Batch(len(wls), 8, "f16", hip_stream=cs, use_graph=False)
    plain = [wrls.Stream(wl.width, wl.height, wl.d, in_dtype="f16", hip_stream=cs) for wl in wls]
    shape = (7, 128)
    b_graph.set_tile(shape[0], shape[1], blocks_per_cu)
    b_plain.set_tile(shape[0], shape[1], blocks_per_cu)
    if blocks_per_cu == 1:
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        assert _tiles(wls, shape) > 2 * cus  # every workgroup loops
    refs = [oracle.Oracle(wl.width, wl.height, wl.d) for wl in wls]
    for t in range(T):
        log("case batch mix blocks_per_cu=%d frame %d" % (blocks_per_cu, t))
        outs_a = [s.step(*dev[i][t]).clone() for i, s in enumerate(alone)]
        outs_g = b_graph.step(mixed, [dev[i][t] for i in range(len(wls))])
        outs_p = b_plain.step(plain, [dev[i][t] for i in range(len(wls))])
        torch.cuda.synchronize()
        for i, wl in enumerate(wls):
            assert torch.equal(outs_a[i], outs_g[i]), (t, wl.name, "graph")
            assert torch.equal(outs_a[i], outs_p[i]), (t, wl.name, "plain")
            f = host[i][t]
            ref = refs[i].step(f.color, f.feats, f.var, f.motion)
            e = g1(outs_g[i].cpu().numpy(), ref, term_scale(refs[i].get_beta(), predictor(f.feats)))
            assert e <= G1_TOL, (t, wl.name, e)


def test_batch_changing_composition_and_empty_steps():
    """Streams join and leave between steps (continuous batching); a stream's
    frames give the same bits whatever shares its launch."""
    import torch
    from paper_2106_08034_amd import wrls
    T = 7
    wls = _mix(0.08, T, n=5)
    dev = [[_dev(f) for f in _frames(wl, T)] for wl in wls]
    alone = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16") for wl in wls]
    ref = [[s.step(*dev[i][t]).clone() for t in range(T)] for i, s in enumerate(alone)]
    b = wrls.Batch(5, 8, "f16")
    mixed = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=b.hip_stream) for wl in wls]
    done = [0] * len(wls)
    schedule = [[0, 1], [0, 1, 2], [], [2, 3, 4], [0, 4], [1, 2, 3, 4, 0], [1], [3], [0, 1, 2, 3, 4],
                [2, 3, 4], [0, 1], [4, 0], [1, 2, 3], [2, 3, 4, 1, 0]]
    for members in schedule:
        members = [i for i in members if done[i] < T]
        outs = b.step([mixed[i] for i in members], [dev[i][done[i]] for i in members])
        torch.cuda.synchronize()
        for i, o in zip(members, outs):
            assert torch.equal(o, ref[i][done[i]]), (i, done[i])
            done[i] += 1
    assert min(done) >= 4


def test_batch_rejects_duplicates_and_mismatches():
    from paper_2106_08034_amd import wrls
    b = wrls.Batch(2, 8, "f16")
    s = wrls.Stream(32, 16, 8, in_dtype="f16", hip_stream=b.hip_stream)
    t32 = wrls.Stream(32, 16, 8, in_dtype="f32", hip_stream=b.hip_stream)
    s10 = wrls.Stream(32, 16, 10, in_dtype="f16", hip_stream=b.hip_stream)
    fr = _dev(_frames(synth.c3(width=32, height=16, frames=1, d=8), 1)[0])
    with pytest.raises(wrls.WrlsError, match="twice"):
        b.step([s, s], [fr, fr])
    with pytest.raises(wrls.WrlsError):
        b.step([t32], [tuple(x.float() for x in fr)])
    with pytest.raises(wrls.WrlsError):
        wrls.wrls_batch_step(b.handle, [s10.handle], [(None, None, None, None, None)])
    with pytest.raises(wrls.WrlsError):
        wrls.wrls_batch_step(b.handle, [s.handle] * 3, [(None,) * 5] * 3)
    assert s.frames == 0


def test_stream_in_caller_memory_equals_library_allocation():
    import torch
    from paper_2106_08034_amd import wrls
    wl = synth.c2(width=150, height=70, frames=5)
    dev = [_dev(f) for f in _frames(wl, 5)]
    p = wrls.make_params(wl.width, wl.height, wl.d)
    need = wrls.wrls_stream_device_bytes(p)
    arena = torch.empty(need // 4 + 64 + 1024, dtype=torch.float32, device="cuda")
    ptr = (arena.data_ptr() + 255) // 256 * 256 + 4096
    a = wrls.Stream(wl.width, wl.height, wl.d)
    b = wrls.Stream(wl.width, wl.height, wl.d, device_mem=(ptr, need))
    for f in dev:
        assert torch.equal(a.step(*f).clone(), b.step(*f).clone())
    b.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [None, (8, 256, 0), (8, 256, 1), (7, 128, -1)])
def test_full_size_c4_mix_batch_equals_alone(shape):
    """The 16-stream mix at its real resolutions (640x480 .. 2560x1440,
    FP16, d = 8) for a few frames: the batched graph replay gives every
    stream the bits of its own launch, with the default tile, with the
    256 x 1 tile the benchmark's autotuner picks, and with persistent grids
    (third entry 1: one workgroup per CU; -1: as many as are resident),
    whose workgroups each loop over dozens of tiles; the smallest stream
    also matches the oracle (G1)."""
    import oracle
    import torch
    from paper_2106_08034_amd import wrls
    T = 3
    wls = _mix(1.0, T)
    log("case c4 full mix %s: " % (shape,) + ", ".join("%dx%d" % (w.width, w.height) for w in wls))
    b = wrls.Batch(len(wls), 8, "f16")
    if shape is not None:
        b.set_tile(*shape)
    small = min(range(len(wls)), key=lambda i: wls[i].width * wls[i].height)
    o = oracle.Oracle(wls[small].width, wls[small].height, 8)
    alone = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=b.hip_stream) for wl in wls]
    mixed = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=b.hip_stream) for wl in wls]
    if shape is not None:
        for s in alone:
            s.set_tile(shape[0], shape[1], 0)
    srcs = [synth.FrameSource(wl) for wl in wls]
    for t in range(T):
        host = [s.next() for s in srcs]
        fr = [_dev(h) for h in host]
        with torch.cuda.stream(torch.cuda.ExternalStream(b.hip_stream)):
            outs_a = [s.step(*fr[i]) for i, s in enumerate(alone)]
            outs_b = b.step(mixed, fr)
        torch.cuda.synchronize()
        for i in range(len(wls)):
            assert torch.equal(outs_a[i], outs_b[i]), (t, wls[i].name)
        if t == T - 1:
            for sa, sb in zip(alone, mixed):
                Pa, Ba = sa.get_state()
                Pb, Bb = sb.get_state()
                assert torch.equal(Pa, Pb) and torch.equal(Ba, Bb)
        h = host[small]
        ref = o.step(h.color, h.feats, h.var, h.motion)
        e = g1(outs_b[small].cpu().numpy(), ref, term_scale(o.get_beta(), predictor(h.feats)))
        log("  frame %d: %s vs oracle G1 %.3g" % (t, wls[small].name, e))
        assert e <= G1_TOL, e


def test_distinct_handles_from_two_host_threads():
    """Distinct handles may be used concurrently: two host threads, each
    stepping its own stream on its own HIP stream, give the bits of the
    same streams run one after the other."""
    import threading

    import torch
    from paper_2106_08034_amd import wrls
    wls = _mix(0.25, 4, n=2)
    frames = [[_dev(f) for f in _frames(wl, 4)] for wl in wls]
    torch.cuda.synchronize()  # the uploads ran on the default stream
    hip = [torch.cuda.Stream(), torch.cuda.Stream()]
    seq_out = []
    for i, wl in enumerate(wls):
        s = wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=hip[i].cuda_stream)
        with torch.cuda.stream(hip[i]):
            outs = [s.step(*f).clone() for f in frames[i]]
        torch.cuda.synchronize()
        seq_out.append(outs)
        s.close()
    par_out = [None, None]
    errors = []

    def run(i):
        try:
            wl = wls[i]
            s = wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=hip[i].cuda_stream)
            with torch.cuda.stream(hip[i]):
                outs = [s.step(*f).clone() for f in frames[i]]
            hip[i].synchronize()
            par_out[i] = outs
            s.close()
        except Exception as e:  # reported below, in the test's thread
            errors.append(e)

    ts = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i in range(2):
        for a, b in zip(seq_out[i], par_out[i]):
            assert torch.equal(a, b)


@pytest.mark.parametrize("d", [1, 2, 4, 7, 9, 10])
@pytest.mark.parametrize("in_dtype", ["f32", "f16"])
def test_batch_every_d_bitwise(d, in_dtype):
    """The batched kernel is compiled per d with its own occupancy hint, and
    d >= 9 gathers two vector groups per batch: at each of these d, three
    streams of different sizes stepped in one batched launch give bitwise
    the outputs and state of the per-frame kernel."""
    import torch
    from paper_2106_08034_amd import wrls
    rng = np.random.default_rng(40 + d)
    sizes = [(70, 9), (131, 5), (64, 12)]
    tdt = torch.float16 if in_dtype == "f16" else torch.float32
    alone = [wrls.Stream(w, h, d, in_dtype=in_dtype) for (w, h) in sizes]
    cs = torch.cuda.current_stream().cuda_stream
    mixed = [wrls.Stream(w, h, d, in_dtype=in_dtype, hip_stream=cs) for (w, h) in sizes]
    b = wrls.Batch(len(sizes), d, in_dtype, hip_stream=cs)
    log("case batch d=%d %s" % (d, in_dtype))
    for t in range(4):
        frames = []
        for (w, h) in sizes:
            color = torch.from_numpy(rng.uniform(0, 1.5, (3, h, w)).astype(np.float32)).cuda().to(tdt)
            feats = torch.from_numpy(rng.uniform(0, 1, (d - 1, h, w)).astype(np.float32)).cuda().to(tdt)
            var = torch.from_numpy(np.exp(-3 + rng.standard_normal((h, w))).astype(np.float32)).cuda()
            mot = torch.from_numpy(rng.uniform(-1.6, 1.6, (2, h, w)).astype(np.float32)).cuda()
            frames.append((color, feats if d > 1 else None, var, mot))
        outs = b.step(mixed, frames)
        for k, (s, f) in enumerate(zip(alone, frames)):
            assert torch.equal(s.step(*f), outs[k]), (d, in_dtype, t, k)
    for s, m in zip(alone, mixed):
        P0, B0 = s.get_state()
        P1, B1 = m.get_state()
        assert torch.equal(P0, P1) and torch.equal(B0, B1)
    b.close()
    torch.cuda.synchronize()
