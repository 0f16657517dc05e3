"""Serving loop for many concurrent denoising sessions on one GPU.

Each session (a viewer) owns a wRLS stream whose state stays resident in
HBM for the session's lifetime.  Sessions are admitted while their device
footprint fits a fixed HBM budget (an arena carved once from device memory,
so admission never allocates); the others wait in arrival order.  Frames
arrive per session at its frame rate; every tick the scheduler packs the
sessions' due frames (oldest first, at most max_batch) into one batched step
(continuous batching: sessions join and leave between steps), which goes out
at once, on one of two HIP streams, with up to 2 * max_batch launches in
flight.  A session has at most one frame in flight, which orders its frames
without cross-stream waits and lets the launches overlap on the device.
Latency is measured on the host from a frame's arrival to the moment its
step is seen complete.

A batch of one frame goes out as a plain wrls_step launch: the batched
step's table staging and graph replay would only add latency to it.

The per-stream baseline serves the same trace with one wrls_step launch per
ready frame (no batching), alternating between the same two HIP streams,
with the same number of launches in flight.

The scheduling rules (arena, admission, batch composition) are plain
Python, independent of the GPU; Server drives them against the library.
"""
from __future__ import annotations

import bisect
import dataclasses
import time
from typing import Dict, List, Optional, Sequence, Tuple

ALIGN = 256

# The saturating variant of the 32-session serving trace: arrivals at 16/s
# instead of 4/s and frame rates of 120-240 Hz instead of 30-60, which offers
# 11-17 Gpx/s from t = 3 s on, more than one GPU steps at d = 8 with FP16
# inputs (keyword arguments of synth.c5_sessions).
SATURATING = dict(rate=16.0, fps_range=(120.0, 240.0))

# A launch-bound variant: the same 32 sessions at small resolutions and high
# frame rates (8.5-10 thousand frames per second in all from t = 3 s on,
# 1.2-1.5 Gpx/s): here the cost per launch, not the GPU's bandwidth, decides
# what a server delivers.
SMALL_FRAMES = dict(rate=16.0, resolutions=((320, 240), (480, 270), (640, 360)),
                    fps_range=(240.0, 480.0))


class Arena:
    """First-fit allocator of byte ranges in [0, size), ALIGN-aligned, with
    coalescing of free neighbours."""

    def __init__(self, size: int):
        self.size = size
        self.free: List[Tuple[int, int]] = [(0, size)]  # sorted (offset, length)
        self.used: Dict[int, int] = {}

    @staticmethod
    def round_up(n: int) -> int:
        return (n + ALIGN - 1) // ALIGN * ALIGN

    def alloc(self, nbytes: int) -> Optional[int]:
        n = self.round_up(max(1, nbytes))
        for i, (off, length) in enumerate(self.free):
            if length >= n:
                if length == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, length - n)
                self.used[off] = n
                return off
        return None

    def release(self, off: int):
        n = self.used.pop(off)
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        # merge with the right neighbour, then the left one
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (off, n + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)

    @property
    def bytes_used(self) -> int:
        return sum(self.used.values())


@dataclasses.dataclass
class SessionState:
    sid: int
    width: int
    height: int
    fps: float
    arrival: float
    end: float
    admitted_at: Optional[float] = None
    next_frame: int = 0           # index of the next frame to submit
    in_flight: bool = False
    finished: bool = False
    offset: Optional[int] = None  # arena offset of its state and output
    latencies: List[float] = dataclasses.field(default_factory=list)

    def frame_time(self, k: int) -> float:
        """Arrival time of frame k (frames start when the session is admitted)."""
        return self.admitted_at + k / self.fps

    def ready(self, now: float) -> bool:
        return (self.admitted_at is not None and not self.finished and not self.in_flight
                and self.frame_time(self.next_frame) <= now
                and self.frame_time(self.next_frame) < self.end)


class Scheduler:
    """Admission by device footprint (and optionally by pixel rate) and batch
    composition (no GPU).  rate_budget: pixels per second the admitted
    sessions may offer together (their width x height x frame rate); None
    admits by memory alone, so an offered load above the GPU's rate queues
    frames without bound."""

    def __init__(self, budget: int, footprint, max_batch: int, rate_budget: Optional[float] = None):
        self.arena = Arena(budget)
        self.footprint = footprint      # (width, height) -> bytes
        self.max_batch = max_batch
        self.rate_budget = rate_budget
        self.rate = 0.0                 # pixels per second the active sessions offer
        self.waiting: List[SessionState] = []
        self.active: List[SessionState] = []
        self.done: List[SessionState] = []
        self.rejected: List[SessionState] = []

    @staticmethod
    def offered(s: SessionState) -> float:
        return float(s.width * s.height) * s.fps

    def arrive(self, s: SessionState):
        too_fast = self.rate_budget is not None and self.offered(s) > self.rate_budget
        if self.footprint(s.width, s.height) > self.arena.size or too_fast:
            self.rejected.append(s)       # can never fit
        else:
            self.waiting.append(s)

    def admit(self, now: float) -> List[SessionState]:
        """Admits waiting sessions in arrival order while they fit (memory,
        and the pixel rate when it is budgeted)."""
        admitted = []
        while self.waiting:
            s = self.waiting[0]
            if self.rate_budget is not None and self.rate + self.offered(s) > self.rate_budget:
                break                     # head-of-line: keep arrival order
            off = self.arena.alloc(self.footprint(s.width, s.height))
            if off is None:
                break
            self.waiting.pop(0)
            self.rate += self.offered(s)
            s.offset = off
            s.admitted_at = now
            s.end = now + (s.end - s.arrival)   # a session lasts its duration once served
            self.active.append(s)
            admitted.append(s)
        return admitted

    def next_batch(self, now: float) -> List[SessionState]:
        """The sessions whose next frame is due and that have none in flight,
        oldest due frame first, at most max_batch."""
        ready = [s for s in self.active if s.ready(now)]
        ready.sort(key=lambda s: s.frame_time(s.next_frame))
        return ready[: self.max_batch]

    def next_launches(self, now: float, per_stream: bool, slots: int) -> List[List[SessionState]]:
        """The launches to issue now, given `slots` free launch slots, for the
        sessions of next_batch(now): per stream, one launch per session;
        batched, one launch per resolution among them (in order of each
        resolution's oldest due frame).  A batched launch completes all its
        frames together, so a small frame batched with a large one would
        wait for it; frames of one size finish together either way.  At
        most `slots` launches."""
        if slots <= 0:
            return []
        members = self.next_batch(now)
        if per_stream:
            return [[s] for s in members[:slots]]
        groups: Dict[Tuple[int, int], List[SessionState]] = {}
        for s in members:
            groups.setdefault((s.width, s.height), []).append(s)
        return list(groups.values())[:slots]

    def retire(self, now: float) -> List[SessionState]:
        """Ends sessions past their end with nothing in flight; frees memory."""
        gone = [s for s in self.active
                if not s.in_flight and s.frame_time(s.next_frame) >= s.end and now >= s.end]
        for s in gone:
            s.finished = True
            self.active.remove(s)
            self.arena.release(s.offset)
            self.rate -= self.offered(s)
            self.done.append(s)
        return gone


def percentile(xs: Sequence[float], q: float) -> float:
    if not xs:
        return float("nan")
    ys = sorted(xs)
    k = (len(ys) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(ys) - 1)
    return ys[lo] + (ys[hi] - ys[lo]) * (k - lo)


class Server:
    """Runs a session workload in real time on the GPU."""

    def __init__(self, budget_bytes: int, d: int = 8, in_dtype: str = "f16", max_batch: int = 32,
                 lam: float = 0.98, tile: Optional[Tuple[int, int, int]] = None,
                 per_stream: bool = False, rate_budget: Optional[float] = None):
        """per_stream: serve with one wrls_step launch per frame (the
        unbatched baseline) instead of batched steps.  rate_budget: admit
        sessions only while their offered pixels per second fit it (None:
        by memory alone)."""
        import torch

        from . import wrls
        self.torch, self.wrls = torch, wrls
        self.d, self.in_dtype, self.lam = d, in_dtype, lam
        self.per_stream = per_stream
        # launches in flight, batched or not: two per batch slot, so that a
        # due frame never waits on the host for the GPU to finish others
        self.max_inflight = 2 * max_batch
        self.arena_mem = torch.empty(budget_bytes + ALIGN, dtype=torch.uint8, device="cuda")
        self.delta = (-self.arena_mem.data_ptr()) % ALIGN   # first aligned byte
        # two HIP streams (torch's, which outlive every context), and enough
        # batch contexts on them that each in-flight launch has its own frame
        # table (a context holds two): a new batched step never waits for a
        # table to come free
        self.hip = [torch.cuda.Stream(), torch.cuda.Stream()]
        self.batches = [wrls.Batch(max_batch, d, in_dtype, hip_stream=self.hip[k % 2].cuda_stream)
                        for k in range(self.max_inflight // 2)]
        if tile is not None:
            for b in self.batches:
                b.set_tile(*tile)
        # handles are created on hip[0]; closed after moving them to an idle
        # stream (their work is complete by then, so the close need not wait)
        self.idle = torch.cuda.Stream()
        self.sched = Scheduler(budget_bytes, self.footprint, max_batch, rate_budget)
        # single-frame launches use the batch's tile shape too
        self.stream_tile = tile
        self.streams: Dict[int, object] = {}
        self.outs: Dict[int, object] = {}
        self.created: Dict[int, object] = {}   # sid -> event after its initialisation

    def close(self):
        """Releases the arena and the batch contexts (a Server's scheduler
        refers back to it, so it is not freed by reference counting alone)."""
        for sid in list(self.streams):
            h = self.streams.pop(sid)
            self.wrls.wrls_set_hip_stream(h.handle, self.idle.cuda_stream)
            h.close()
        self.outs.clear()
        self.created.clear()
        for b in self.batches:
            b.close()
        self.batches = []
        self.arena_mem = None
        self.sched = None

    def footprint(self, width: int, height: int) -> int:
        """Device bytes a session holds: both state copies and its output."""
        p = self.wrls.make_params(width, height, self.d, lam=self.lam, in_dtype=self.in_dtype)
        return (Arena.round_up(self.wrls.wrls_stream_device_bytes(p))
                + Arena.round_up(3 * width * height * 4))

    def _open(self, s: SessionState):
        torch, wrls = self.torch, self.wrls
        p = wrls.make_params(s.width, s.height, self.d, lam=self.lam, in_dtype=self.in_dtype)
        nstate = Arena.round_up(wrls.wrls_stream_device_bytes(p))
        start = self.delta + s.offset
        ptr = self.arena_mem.data_ptr() + start
        self.streams[s.sid] = wrls.Stream(s.width, s.height, self.d, lam=self.lam,
                                          in_dtype=self.in_dtype,
                                          hip_stream=self.hip[0].cuda_stream,
                                          device_mem=(ptr, nstate))
        if self.stream_tile is not None:
            self.streams[s.sid].set_tile(self.stream_tile[0], self.stream_tile[1], 0)
        ev = torch.cuda.Event()
        ev.record(self.hip[0])
        self.created[s.sid] = ev
        n = 3 * s.width * s.height * 4
        self.outs[s.sid] = self.arena_mem[start + nstate: start + nstate + n] \
            .view(torch.float32).view(3, s.height, s.width)

    def _close(self, s: SessionState):
        h = self.streams.pop(s.sid)
        self.wrls.wrls_set_hip_stream(h.handle, self.idle.cuda_stream)
        h.close()
        self.outs.pop(s.sid)
        self.created.pop(s.sid, None)

    def run(self, sessions, frame_pools, seconds: float, record: Optional[int] = None,
            poll: float = 0.0, record_frames: Optional[int] = None):
        """sessions: synth.Session list; frame_pools[(w, h)]: list of device
        frame tuples, cycled.  Runs until `seconds` have passed or every
        session is served.  record: sid whose outputs are kept (host copies)
        for the alone-vs-mix and oracle checks, its first record_frames
        frames (None: all).  poll: seconds to sleep when a pass launched
        nothing; 0 (the default) polls without sleeping, since a sleep adds
        its granularity (0.1-0.3 ms here) to every frame's latency."""
        torch = self.torch
        pending = sorted([SessionState(x.sid, x.width, x.height, x.fps, x.arrival,
                                       x.arrival + x.duration) for x in sessions],
                         key=lambda x: x.arrival)
        inflight = []          # (event, members, pixels)
        recorded = []
        steps = 0
        nbatched = 0           # batched launches so far
        pixels = 0
        max_active = 0
        t0 = time.perf_counter()

        def complete(entry, t_done):
            nonlocal pixels
            _, members, npx = entry
            for s in members:
                s.latencies.append(t_done - s.frame_time(s.next_frame - 1))
                s.in_flight = False
                if s.sid == record and (record_frames is None or len(recorded) < record_frames):
                    recorded.append(self.outs[s.sid].cpu())
            pixels += npx

        while True:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                self.sched.arrive(pending.pop(0))
            for s in self.sched.admit(now):
                self._open(s)
            max_active = max(max_active, len(self.sched.active))
            still = []
            for entry in inflight:
                if entry[0].query():
                    complete(entry, time.perf_counter() - t0)
                else:
                    still.append(entry)
            inflight = still
            for s in self.sched.retire(now):
                self._close(s)
            if now >= seconds or (not pending and not self.sched.active and not self.sched.waiting
                                  and not inflight):
                break
            launches = self.sched.next_launches(now, self.per_stream,
                                                self.max_inflight - len(inflight))
            for members in launches:
                batched = not self.per_stream and len(members) > 1
                if batched:   # the next context; it runs on its own stream
                    ctx = self.batches[nbatched % len(self.batches)]
                    bi = (nbatched % len(self.batches)) % 2
                    nbatched += 1
                else:
                    bi = steps % 2
                for s in members:   # a new session's initialisation ran on hip[0]
                    ev = self.created.pop(s.sid, None)
                    if ev is not None and bi != 0:
                        self.hip[bi].wait_event(ev)
                frames = []
                for s in members:
                    pool = frame_pools[(s.width, s.height)]
                    frames.append(pool[s.next_frame % len(pool)])
                if batched:
                    ctx.step([self.streams[s.sid] for s in members], frames,
                             [self.outs[s.sid] for s in members])
                else:
                    st = self.streams[members[0].sid]
                    self.wrls.wrls_set_hip_stream(st.handle, self.hip[bi].cuda_stream)
                    st.step(*frames[0], out=self.outs[members[0].sid])
                ev = torch.cuda.Event()
                ev.record(self.hip[bi])
                for s in members:
                    s.in_flight = True
                    s.next_frame += 1
                inflight.append((ev, members, sum(s.width * s.height for s in members)))
                steps += 1
            if launches:
                continue
            time.sleep(poll)
        for entry in inflight:
            entry[0].synchronize()
            complete(entry, time.perf_counter() - t0)
        wall = time.perf_counter() - t0
        for s in list(self.sched.active):
            s.end = 0.0
        for s in self.sched.retire(float("inf")):
            self._close(s)
        lat = [x for s in self.sched.done for x in s.latencies]
        waits = [s.admitted_at - s.arrival for s in self.sched.done if s.admitted_at is not None]
        return {
            "mode": "per_stream_launches" if self.per_stream else "batched",
            "seconds": round(wall, 3),
            "steps": steps,
            "frames": len(lat),
            "mean_batch": round(len(lat) / max(1, steps), 2),
            "mpix_per_s": round(pixels / wall / 1e6, 2),
            "p50_ms": round(percentile(lat, 50) * 1e3, 3),
            "p99_ms": round(percentile(lat, 99) * 1e3, 3),
            "max_ms": round(max(lat) * 1e3, 3) if lat else None,
            "sessions_served": sum(1 for s in self.sched.done if s.latencies),
            "sessions_waiting_at_end": len(self.sched.waiting),
            "sessions_rejected": len(self.sched.rejected),
            "max_concurrent": max_active,
            "rate_budget_gpx_s": (round(self.sched.rate_budget / 1e9, 3)
                                  if self.sched.rate_budget is not None else None),
            # arrival to admission: grows when the HBM budget makes sessions queue
            "admission_wait_p50_ms": round(percentile(waits, 50) * 1e3, 3) if waits else None,
            "admission_wait_max_ms": round(max(waits) * 1e3, 3) if waits else None,
        }, recorded
