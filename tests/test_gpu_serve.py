"""The serving loop on the GPU: sessions admitted by HBM footprint, frames
continuously batched with two steps in flight; a session's outputs are
bitwise those of the same session run alone, and match the FP64 oracle."""
import pytest
import torch

import synth
from parity import G1_TOL, g1, log, predictor, term_scale, to_dev

pytestmark = pytest.mark.gpu


def _pools(shapes, count=3, host=None):
    pools = {}
    for i, (w, h) in enumerate(shapes):
        src = synth.FrameSource(synth.c5_frame_pool(w, h, count), stream=i)
        frames = [src.next() for _ in range(count)]
        if host is not None:
            host[(w, h)] = frames
        pools[(w, h)] = [tuple(to_dev(a) for a in (f.color, f.feats, f.var, f.motion)) for f in frames]
    return pools


def _replay_alone(sess, pool, n):
    from paper_2106_08034_amd import wrls
    s = wrls.Stream(sess.width, sess.height, 8, in_dtype="f16")
    outs = [s.step(*pool[k % len(pool)]).cpu() for k in range(n)]
    s.close()
    return outs


@pytest.mark.parametrize("per_stream", [False, True])
def test_served_session_equals_alone_bitwise(per_stream):
    """Batched serving (one-frame batches go out as plain launches) and the
    per-stream baseline: a session's outputs are those of the session run
    alone, bitwise, and match the oracle."""
    from paper_2106_08034_amd.serve import Server
    shapes = [(160, 96), (224, 128), (96, 64)]
    sessions = [synth.Session(sid=i, width=shapes[i % 3][0], height=shapes[i % 3][1],
                              fps=60.0 + 10 * i, arrival=0.05 * i, duration=0.6 + 0.1 * i)
                for i in range(8)]
    host = {}
    pools = _pools(shapes, host=host)
    srv = Server(budget_bytes=256 << 20, max_batch=8, per_stream=per_stream)
    log("case serve 8 small sessions, per_stream=%s" % per_stream)
    res, rec = srv.run(sessions, pools, seconds=5.0, record=3)
    log("serve result %s" % res)
    assert res["sessions_served"] == 8 and res["frames"] > 100
    assert len(rec) >= 20
    assert res["mode"] == ("per_stream_launches" if per_stream else "batched")
    if per_stream:
        assert res["steps"] == res["frames"]   # one launch per frame
    key = (sessions[3].width, sessions[3].height)
    alone = _replay_alone(sessions[3], pools[key], len(rec))
    for k, (a, b) in enumerate(zip(alone, rec)):
        assert torch.equal(a, b), k
    # the served session against the FP64 oracle, frame by frame (the pool
    # cycles, as it did for the server)
    import oracle
    o = oracle.Oracle(key[0], key[1], 8)
    worst = 0.0
    for k, out in enumerate(rec):
        f = host[key][k % len(host[key])]
        ref = o.step(f.color, f.feats, f.var, f.motion)
        e = g1(out.numpy(), ref, term_scale(o.get_beta(), predictor(f.feats)))
        worst = max(worst, e)
        assert e <= G1_TOL, (k, e)
    log("served session vs oracle over %d frames: worst G1 %.3g" % (len(rec), worst))
    srv.close()


def test_budget_admission_queues_sessions():
    from paper_2106_08034_amd.serve import Server
    shapes = [(256, 160)]
    sessions = [synth.Session(sid=i, width=256, height=160, fps=100.0, arrival=0.0, duration=0.3)
                for i in range(5)]
    pools = _pools(shapes)
    srv = Server(budget_bytes=1, max_batch=8)
    one = srv.footprint(256, 160)
    srv = Server(budget_bytes=2 * one, max_batch=8)   # two sessions fit at a time
    log("case serve with a 2-session budget")
    res, _ = srv.run(sessions, pools, seconds=10.0)
    log("serve result %s" % res)
    assert res["max_concurrent"] == 2
    assert res["sessions_served"] == 5 and res["sessions_waiting_at_end"] == 0
