"""Serving logic without a GPU: arena allocation, admission by footprint,
batch composition, retirement."""
import pytest

import synth
from paper_2106_08034_amd.serve import ALIGN, SATURATING, Arena, Scheduler, SessionState, percentile


def test_arena_first_fit_alignment_and_coalescing():
    a = Arena(10 * ALIGN)
    x = a.alloc(1)
    y = a.alloc(ALIGN + 1)
    z = a.alloc(3 * ALIGN)
    assert (x, y, z) == (0, ALIGN, 3 * ALIGN)
    assert all(o % ALIGN == 0 for o in (x, y, z))
    assert a.alloc(5 * ALIGN) is None          # only 4 * ALIGN left at the end
    a.release(y)
    assert a.alloc(3 * ALIGN) == 6 * ALIGN      # first fit skips the 2-ALIGN hole
    a.release(x)
    assert a.free[0] == (0, 3 * ALIGN)          # x and y's holes merged
    a.release(z)
    a.release(6 * ALIGN)
    assert a.free == [(0, 10 * ALIGN)] and a.bytes_used == 0


def _sess(sid, w=100, h=50, fps=50.0, arrival=0.0, dur=1.0):
    return SessionState(sid, w, h, fps, arrival, arrival + dur)


def test_admission_by_footprint_in_arrival_order():
    fp = lambda w, h: w * h * 100
    sch = Scheduler(budget=1_200_000, footprint=fp, max_batch=8)
    big = _sess(0, 100, 100)      # 1.0 MB
    small = _sess(1, 10, 10)      # 10 kB
    huge = _sess(2, 200, 100)     # 2 MB: can never fit
    for s in (big, small, huge):
        sch.arrive(s)
    assert sch.rejected == [huge]
    assert [s.sid for s in sch.admit(0.0)] == [0, 1]
    late = _sess(3, 100, 50)      # 0.5 MB: waits for memory
    sch.arrive(late)
    assert sch.admit(0.1) == [] and sch.waiting == [late]
    big.next_frame = 1000          # past its end
    assert [s.sid for s in sch.retire(10.0)] == [0]
    assert [s.sid for s in sch.admit(10.0)] == [3]
    assert late.admitted_at == 10.0


def test_batch_composition_one_frame_in_flight_and_due_frames():
    sch = Scheduler(budget=10 ** 9, footprint=lambda w, h: 1000, max_batch=2)
    a, b, c = _sess(0, fps=10), _sess(1, fps=100), _sess(2, fps=100)
    for s in (a, b, c):
        sch.arrive(s)
    sch.admit(0.0)
    assert len(sch.active) == 3
    assert [s.sid for s in sch.next_batch(0.0)] == [0, 1]      # max_batch caps the step
    a.in_flight = True
    assert [s.sid for s in sch.next_batch(0.0)] == [1, 2]
    a.in_flight = False
    a.next_frame = 1               # next frame of a due at 0.1 s
    b.next_frame = 3               # due at 0.03 s
    c.next_frame = 2               # due at 0.02 s: the oldest goes first
    assert [s.sid for s in sch.next_batch(0.05)] == [2, 1]
    c.next_frame = 9               # due at 0.09 s
    assert [s.sid for s in sch.next_batch(0.1)] == [1, 2]
    b.in_flight = True
    assert [s.sid for s in sch.next_batch(0.1)] == [2, 0]


def test_sessions_workload_is_seeded_and_shaped():
    s1, s2 = synth.c5_sessions(), synth.c5_sessions()
    assert s1 == s2 and len(s1) == 32
    assert all((x.width, x.height) in synth.C5_RESOLUTIONS for x in s1)
    assert all(30.0 <= x.fps <= 60.0 for x in s1)
    arr = [x.arrival for x in s1]
    assert arr == sorted(arr) and arr[0] == 0.0
    # Poisson(4/s): 31 gaps with mean about 1/4 s
    assert 0.1 < (arr[-1] / 31) < 0.5


def test_percentile():
    assert percentile([3, 1, 2], 50) == 2
    assert percentile([1, 2, 3, 4], 100) == 4
    assert percentile(list(range(101)), 99) == pytest.approx(99)


def test_launches_batched_against_per_stream():
    """The per-stream baseline issues one launch per due frame, the same
    frames in the same order as the batched step, within its free launch
    slots; the batched mode issues one launch, or none without a free slot."""
    sch = Scheduler(budget=10 ** 9, footprint=lambda w, h: 1000, max_batch=3)
    ss = [_sess(i, fps=100) for i in range(4)]
    for s in ss:
        sch.arrive(s)
    sch.admit(0.0)
    ss[1].next_frame = 1           # due at 0.01 s: after the others
    batched = sch.next_launches(0.02, per_stream=False, slots=1)
    assert [[s.sid for s in m] for m in batched] == [[0, 2, 3]]
    assert sch.next_launches(0.02, per_stream=False, slots=0) == []
    single = sch.next_launches(0.02, per_stream=True, slots=8)
    assert [[s.sid for s in m] for m in single] == [[0], [2], [3]]
    assert [[s.sid for s in m] for m in sch.next_launches(0.02, True, 2)] == [[0], [2]]
    for s in ss:
        s.in_flight = True
    assert sch.next_launches(0.02, True, 8) == [] and sch.next_launches(0.02, False, 2) == []


def test_saturating_trace_offers_more_than_the_step_rate():
    """The saturating variant of the serving trace (arrivals at 16/s, frame
    rates 120-240 Hz) offers more pixels per second from t = 3 s on than one
    GPU steps at d = 8 FP16 (about 10 Gpx/s measured); the plain trace offers
    at most about 4 Gpx/s."""
    def offered(sessions, t):
        return sum(s.width * s.height * s.fps for s in sessions if s.arrival <= t < s.arrival + s.duration)
    plain = synth.c5_sessions()
    sat = synth.c5_sessions(**SATURATING)
    assert min(offered(sat, t) for t in (3, 5, 8, 10)) > 11e9
    assert max(offered(plain, t) for t in range(16)) < 4.5e9


def test_batched_launches_group_by_resolution():
    """Batched, the due frames go out as one launch per resolution, in the
    order of each resolution's oldest due frame, within the free slots."""
    sch = Scheduler(budget=10 ** 9, footprint=lambda w, h: 1000, max_batch=8)
    ss = [_sess(0, 100, 50, fps=100), _sess(1, 200, 100, fps=100), _sess(2, 100, 50, fps=100),
          _sess(3, 300, 100, fps=100), _sess(4, 200, 100, fps=100)]
    for s in ss:
        sch.arrive(s)
    sch.admit(0.0)
    ss[0].next_frame = 2           # due at 0.02 s, after the others (0.01 s)
    for s in ss[1:]:
        s.next_frame = 1
    got = [[s.sid for s in m] for m in sch.next_launches(0.03, per_stream=False, slots=8)]
    assert got == [[1, 4], [2, 0], [3]]
    assert [[s.sid for s in m] for m in sch.next_launches(0.03, False, 2)] == [[1, 4], [2, 0]]
    assert len(sch.next_launches(0.03, True, 8)) == 5


def test_admission_by_pixel_rate():
    """With a pixel-rate budget, a session is admitted only while the
    admitted sessions' width x height x fps stays within it (arrival order
    kept); retiring a session frees its rate; a session offering more than
    the whole budget is rejected."""
    sch = Scheduler(budget=10 ** 12, footprint=lambda w, h: 1000, max_batch=8, rate_budget=3.0e6)
    a = _sess(0, 100, 100, fps=100)      # 1.0 Mpx/s
    b = _sess(1, 100, 100, fps=150)      # 1.5 Mpx/s
    c = _sess(2, 100, 100, fps=100)      # 1.0 Mpx/s: waits for a or b
    d = _sess(3, 100, 100, fps=10)       # 0.1 Mpx/s: fits, but waits behind c
    huge = _sess(4, 200, 200, fps=100)   # 4.0 Mpx/s: never fits
    for s in (a, b, c, d, huge):
        sch.arrive(s)
    assert sch.rejected == [huge]
    assert [s.sid for s in sch.admit(0.0)] == [0, 1]
    assert sch.rate == pytest.approx(2.5e6)
    a.next_frame = 1000
    assert [s.sid for s in sch.retire(10.0)] == [0]
    assert sch.rate == pytest.approx(1.5e6)
    assert [s.sid for s in sch.admit(10.0)] == [2, 3]
    assert sch.rate == pytest.approx(2.6e6)
