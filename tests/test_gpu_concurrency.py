"""Distinct stream handles share no state: streams stepped (and blended)
concurrently, from several host threads onto several HIP streams at once,
give bitwise the results of the same streams stepped one after another.
The handles' only shared resources are the device and the library's code;
this checks that no kernel or host path keeps per-library state that a
concurrent call could disturb."""
import threading

import numpy as np
import pytest

import synth
from parity import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    yield


CASES = [("c2", dict(width=197, height=83), "invvar", "f32"),
         ("c3", dict(width=203, height=117), "invvar", "f16"),
         ("c2", dict(width=160, height=45), "paper", "f32"),
         ("c3", dict(width=96, height=64), "one", "f16"),
         ("c2", dict(width=320, height=240), "invvar", "f32"),
         ("c3", dict(width=131, height=7), "invvar", "f16")]
T = 5


def _inputs():
    runs = []
    for k, (scene, size, mode, dt) in enumerate(CASES):
        wl = (synth.c2 if scene == "c2" else synth.c3)(frames=T, **size)
        src = synth.FrameSource(wl)
        frames = []
        for _ in range(T):
            f = src.next()
            frames.append(tuple(to_dev(a) for a in (f.color, f.feats, f.var, f.motion)))
        d = 4 if mode == "paper" else wl.d
        runs.append((wl, d, mode, dt, frames))
    return runs


def _run_one(wrls, run, hip_stream, results, key):
    wl, d, mode, dt, frames = run
    s = wrls.Stream(wl.width, wl.height, d, in_dtype=dt, weight_mode=mode, hip_stream=hip_stream)
    outs = []
    for c, fe, v, m in frames:
        fe = None if mode == "paper" else fe
        v = v if mode == "invvar" else None
        out = s.step(c, fe, v, m)
        fin = s.blend(fe, out, 1.5, 0.15)
        outs += [out, fin]
    P, B = s.get_state()
    results[key] = (outs, P, B, s)


def test_concurrent_streams_equal_sequential():
    import torch
    from paper_2106_08034_amd import wrls
    runs = _inputs()
    # sequential: every stream on the default stream, one after another
    seq = {}
    for k, run in enumerate(runs):
        _run_one(wrls, run, None, seq, k)
    torch.cuda.synchronize()
    ref = {k: ([o.cpu() for o in v[0]], v[1].cpu(), v[2].cpu()) for k, v in seq.items()}
    for v in seq.values():
        v[3].close()
    # concurrent: one host thread per stream, on three HIP streams
    hips = [torch.cuda.Stream() for _ in range(3)]
    for rep in range(2):
        got, errors = {}, []

        def work(k):
            try:
                _run_one(wrls, runs[k], hips[k % 3].cuda_stream, got, k)
            except Exception as e:  # reported below
                errors.append((k, repr(e)))

        threads = [threading.Thread(target=work, args=(k,)) for k in range(len(runs))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        assert not errors, errors
        for k in range(len(runs)):
            outs, P, B, s = got[k]
            r_outs, r_P, r_B = ref[k]
            same = all(torch.equal(a.cpu(), b) for a, b in zip(outs, r_outs))
            same = same and torch.equal(P.cpu(), r_P) and torch.equal(B.cpu(), r_B)
            log("concurrent rep %d case %d (%s %s %s): %s" % (rep, k, CASES[k][0], CASES[k][2],
                                                            CASES[k][3], "bitwise" if same else "DIFFERS"))
            assert same, (rep, k)
            s.close()
    torch.cuda.synchronize()
