"""Autotuner for the launch shape of the wRLS kernels.

The per-frame kernel takes a tile shape (tile width, workgroup size, tile
order) and the batched persistent kernel additionally a grid size
(workgroups per compute unit).  The best choice depends on the device, the
predictor length d, the input type and the image size, and is found by
timing: each candidate runs a few frames of the caller's workload on scratch
streams (the caller's streams are not advanced) and the fastest median
wins.  Results are cached in a JSON file keyed by device, kind, d, input
type and resolution class, so a workload is tuned once per machine.
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Dict, List, Optional, Sequence, Tuple

from . import wrls

# (tile_w_log2, block_threads) candidates: 32..256-pixel-wide tiles of
# 128- and 256-thread workgroups (64-lane wavefronts).
TILE_CANDIDATES: Tuple[Tuple[int, int], ...] = ((5, 128), (6, 128), (7, 128), (5, 256), (6, 256),
                                               (7, 256), (8, 256))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "wrls_mi355x", "autotune.json")


def resolution_class(pixels: int) -> str:
    """Coarse image-size bucket the tuned shape is reused for."""
    for name, bound in (("<=0.5M", 0.5e6), ("<=1.5M", 1.5e6), ("<=4M", 4.0e6)):
        if pixels <= bound:
            return name
    return ">4M"


class TuneCache:
    """JSON file of tuned shapes; concurrent writers keep the last write."""

    def __init__(self, path: Optional[str] = DEFAULT_CACHE):
        self.path = path
        self.data: Dict[str, dict] = {}
        if path and os.path.exists(path):
            try:
                with open(path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    @staticmethod
    def key(device: str, kind: str, d: int, in_dtype: str, pixels: int) -> str:
        return "%s|%s|d%d|%s|%s" % (device, kind, d, in_dtype, resolution_class(pixels))

    def get(self, key: str) -> Optional[dict]:
        return self.data.get(key)

    def put(self, key: str, value: dict):
        self.data[key] = value
        if self.path:
            os.makedirs(os.path.dirname(self.path), exist_ok=True)
            tmp = self.path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s/%s/%dCU" % (p.name, getattr(p, "gcnArchName", "?"), p.multi_processor_count)


def _time_steps(step_fn, hip_stream, steps: int, warmup: int) -> float:
    """Median per-step milliseconds of step_fn(i) on hip_stream."""
    import torch
    ext = torch.cuda.ExternalStream(hip_stream) if hip_stream else torch.cuda.current_stream()
    with torch.cuda.stream(ext):
        for i in range(warmup):
            step_fn(i)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(ext)
        for i in range(steps):
            step_fn(warmup + i)
            ev[i + 1].record(ext)
        torch.cuda.synchronize()
    return statistics.median(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))


def tune_stream(width: int, height: int, d: int, frames: Sequence[tuple], in_dtype: str = "f32",
                candidates: Sequence[Tuple[int, int]] = TILE_CANDIDATES, steps: int = 8,
                warmup: int = 2, cache: Optional[TuneCache] = None, force: bool = False):
    """Best (tile_w_log2, block_threads, strip_tiles) for single-stream steps
    on width x height images; frames: device tensors (color, features,
    variance, motion), cycled.  Returns (shape, timings)."""
    cache = cache if cache is not None else TuneCache()
    key = TuneCache.key(_device_name(), "stream", d, in_dtype, width * height)
    hit = cache.get(key)
    if hit and not force:
        return tuple(hit["best"]), hit.get("ms", {})
    import torch
    timings = {}
    for tw, bt in candidates:
        s = wrls.Stream(width, height, d, in_dtype=in_dtype)
        s.set_tile(tw, bt, 0)
        out = torch.empty((3, height, width), device="cuda")
        ms = _time_steps(lambda i: s.step(*frames[i % len(frames)], out=out), s.hip_stream, steps, warmup)
        timings["%dx%d/%d" % (1 << tw, bt >> tw, bt)] = ms
        s.close()
    best_name = min(timings, key=timings.get)
    w, rest = best_name.split("x")
    tw = int(w).bit_length() - 1
    bt = int(rest.split("/")[1])
    best = (tw, bt, 0)
    cache.put(key, {"best": list(best), "ms": timings})
    return best, timings


def tune_batch(shapes: Sequence[Tuple[int, int]], d: int, frames: Sequence[Sequence[tuple]],
               in_dtype: str = "f16", candidates: Sequence[Tuple[int, int]] = TILE_CANDIDATES,
               blocks_per_cu: Sequence[int] = (0, -1), steps: int = 6, warmup: int = 2,
               cache: Optional[TuneCache] = None, force: bool = False):
    """Best (tile_w_log2, block_threads, blocks_per_cu) for batched steps of
    streams with the given (width, height) shapes (blocks_per_cu 0: one
    workgroup per tile, -1: resident persistent grid; see
    wrls_batch_set_tile); frames[i]: device tensors of stream i, cycled.
    Returns (shape, timings)."""
    cache = cache if cache is not None else TuneCache()
    total = sum(w * h for w, h in shapes)
    key = TuneCache.key(_device_name(), "batch%d" % len(shapes), d, in_dtype, total // max(1, len(shapes)))
    hit = cache.get(key)
    if hit and not force:
        return tuple(hit["best"]), hit.get("ms", {})
    import torch
    timings = {}
    b = wrls.Batch(len(shapes), d, in_dtype)
    streams = [wrls.Stream(w, h, d, in_dtype=in_dtype, hip_stream=b.hip_stream) for w, h in shapes]
    outs = [torch.empty((3, h, w), device="cuda") for w, h in shapes]
    for tw, bt in candidates:
        for bpc in blocks_per_cu:
            b.set_tile(tw, bt, bpc)
            ms = _time_steps(lambda i: b.step(streams, [fr[i % len(fr)] for fr in frames], outs),
                             b.hip_stream, steps, warmup)
            timings["%dx%d/%d/bpc%d" % (1 << tw, bt >> tw, bt, bpc)] = ms
    b.close()
    for s in streams:
        s.close()
    best_name = min(timings, key=timings.get)
    tile, bpc = best_name.split("/bpc")
    w, rest = tile.split("x")
    best = (int(w).bit_length() - 1, int(rest.split("/")[1]), int(bpc))
    cache.put(key, {"best": list(best), "ms": timings})
    return best, timings
