#!/usr/bin/env python3
"""Throughput of the wRLS temporal denoiser on one MI355X.

Default workload (the headline): 3840x2160, 30 frames of a camera orbiting
a pivot (per-pixel motion from a seeded depth map), a colour-LUT edit at
frame 15 and a light change at frame 22, d = 10 predictors, FP16 colour and
features, FP32 state, lambda = 0.98, heteroscedastic lognormal noise
variance.  All frames are generated (seeded, synthetic) and uploaded to HBM
before the timed region; one step denoises one frame through the C ABI (one
kernel launch).  Beside the headline the default run also reports:
  parity        the error of a GPU pass from frame 0 against the FP64 oracle's
                outputs of the same frames (the CPU baseline's first pass),
                and against an oracle fed the unrounded FP32 inputs;
  c2            the 1920x1080 d = 8 FP32 pan, with its roofline and parity;
  c4_batched    16 mixed-resolution streams: one batched launch per round
                against 16 per-stream launches;
  serving       32 sessions served with continuous batching against one
                launch per frame, at the trace's load and at a saturating one.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published peak
# MI355X FP32 vector peaks: 157.3 TFLOP/s with packed FP32 instructions,
# which the library's build disables, so 78.6 TFLOP/s is the reachable one.
FP32_VECTOR_PEAK_TFLOPS = 78.6
FP32_PACKED_PEAK_TFLOPS = 157.3
METRIC = "denoised Mpix/s (wRLS step) + % HBM roofline; p99 frame latency @32 streams"
DATA = "synthetic (seeded procedural scene, lognormal per-pixel noise variance)"


def algorithmic_bytes_per_pixel(d: int, in_bytes: int, motion: bool = True) -> int:
    """HBM bytes one pixel-step must move at minimum: inputs (colour 3,
    features d-1 in the input type; variance and motion FP32), the previous
    state read once (d(d+1)/2 + 3d floats), the new state written once, and
    the FP32 output (3 floats)."""
    S = d * (d + 1) // 2 + 3 * d
    inputs = (3 + (d - 1)) * in_bytes + 4 + (8 if motion else 0)
    return inputs + 4 * S + 4 * S + 12


def algorithmic_bytes_per_pixel_paper(in_bytes: int, motion: bool = True) -> int:
    """Paper mode (d = 4, p = [1, z]): colour in the input type, FP32 motion,
    the previous state (P 10, beta 12, history z 3 floats) read once, the new
    state written once, and the FP32 output.  The 3x3 colour neighbourhood of
    the clamp is counted once: its other reads hit the caches."""
    S = 10 + 12 + 3
    return 3 * in_bytes + (8 if motion else 0) + 4 * S + 4 * S + 12


def blend_bytes_per_pixel(d: int, in_bytes: int, paper: bool = False) -> int:
    """The 5x5 spatial blend after a step: the current beta (3d floats) and
    the centre's predictor source (d-1 features in the input type, or the
    3 FP32 history planes in paper mode) read once, the step's output read
    once as the range guide, the blended FP32 output written.  Halo re-reads
    of neighbouring tiles are cache hits and are not counted."""
    pred = 12 if paper else (d - 1) * in_bytes
    return 3 * d * 4 + pred + 12 + 12


def blend_flop_per_pixel(d: int) -> int:
    """Arithmetic of the 5x5 spatial blend per output pixel, counting an FMA
    as 2 flop and exp as 1: for each of the 24 non-centre neighbours the
    bilateral weight (3 colour differences, the squared distance as 1
    multiply and 2 FMAs, the exponent as 1 FMA, exp, the running sum:
    12 flop); for each of the 25 neighbours, 3 channels times d FMAs of the
    weighted coefficient sum; then per channel the dot product with p (d - 1
    FMAs, p_0 = 1) and the normalisation (3 multiplies, 1 division)."""
    return 24 * 12 + 25 * 3 * d * 2 + 3 * (d - 1) * 2 + 4


def measure_copy_gbs(torch, wrls, nbytes: int, reps: int = 10) -> float:
    """Read+write bandwidth of the library's plain copy kernel (16-byte loads,
    non-temporal 16-byte stores) moving nbytes per launch (half read, half
    written), timed with HIP events on the current stream: the measured
    reference beside the 8 TB/s spec."""
    n = max(nbytes // 32 * 4, 1 << 20)  # floats per buffer, a multiple of 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        wrls.wrls_device_copy(b, a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        wrls.wrls_device_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    return gbs


def measure_probe_gbs(torch, stream, frames, reps: int, nbytes: int) -> float:
    """Read+write bandwidth of wrls_traffic_probe on the step's own stream and
    frames: the step's loads and stores (same bytes per launch, same tile
    order and access forms) without the reprojection and the arithmetic,
    timed with HIP events on the current stream.  The stream's state is left
    as it was."""
    tmp = torch.empty((3, stream.H, stream.W), dtype=torch.float32, device="cuda")
    for i in range(3):
        stream.traffic_probe(*frames[i % len(frames)], out=tmp)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for i in range(reps):
        stream.traffic_probe(*frames[i % len(frames)], out=tmp)
    e1.record()
    torch.cuda.synchronize()
    gbs = nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del tmp
    return gbs


def bench_paper_context(args) -> dict:
    """A point shaped like the paper's own timing (Sec. 7.5: the whole
    denoiser -- temporal feature, wRLS with p = [1, z], d = 4, and the 5x5
    blend -- at 1280x720, about 12 ms per frame on a laptop GTX 1070): the
    paper-mode step and the blend per frame at 1280x720, timed over a
    sequence on one HIP stream.  Context only (other hardware, other year,
    synthetic frames), not a target."""
    import torch
    import synth
    from paper_2106_08034_amd import wrls
    wl = synth.c2(width=1280, height=720, frames=8)
    src = synth.FrameSource(wl)
    frames = []
    for _ in range(wl.frames):
        f = src.next()
        frames.append((torch.from_numpy(f.color).cuda(), torch.from_numpy(f.motion).cuda()))
    s = wrls.Stream(wl.width, wl.height, 4, lam=0.98, weight_mode="paper")
    out = torch.empty((3, wl.height, wl.width), device="cuda")
    fin = torch.empty_like(out)
    ss, sr = args.blend_sigmas
    for t in range(3):
        s.step(frames[t][0], None, None, frames[t][1], out=out)
        s.blend(None, out, ss, sr, out=fin)
    K = 30
    cs = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(cs)
    for t in range(K):
        c, m = frames[(3 + t) % wl.frames]
        s.step(c, None, None, m, out=out)
        s.blend(None, out, ss, sr, out=fin)
    e1.record(cs)
    torch.cuda.synchronize()
    s.close()
    ms = e0.elapsed_time(e1) / K
    return {"workload": "1280x720, paper mode (d = 4, temporal feature, Eq. 13 weight) + 5x5 blend, "
                        "step and blend per frame",
            "ms_per_frame": round(ms, 4),
            "paper": {"ms_per_frame": 12.0, "plus_minus_ms": 2.5,
                      "hardware": "Nvidia GTX 1070 (laptop), whole denoiser, Sec. 7.5"},
            "note": "context only: different hardware, year and inputs; not a target"}


def kernel_source_hash() -> str:
    """Identifies the code that shapes a launch's memory traffic: the kernels,
    the internal header whose constants they compile with, and the host side
    that lays out the state (plane pitch) and launches them."""
    h = hashlib.sha256()
    for f in ("wrls_kernels.hip", "wrls_internal.h", "wrls_api.hip"):
        h.update(open(os.path.join(ROOT, "paper_2106_08034_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str = ""):
    """HBM traffic per launch from the committed rocprofv3 counter summary
    (kernel "" = the step kernel, "blend" = the spatial blend), if it was
    taken on the current kernel source."""
    name = "traffic_%s%s.json" % (kernel + "_" if kernel else "", workload)
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    """The host CPU's model name (lscpu), with its family, model and stepping
    numbers (a virtual machine may report only a generic name), and the
    host's logical CPU count, for the CPU baseline."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f[k.strip()] = v.strip()
        name = f.get("Model name", "unknown")
        ids = ", ".join("%s %s" % (k.lower(), f[k]) for k in ("CPU family", "Model", "Stepping") if k in f)
        return "%s (%s; %s logical CPUs)" % (name, ids, f.get("CPU(s)", "?"))
    except (OSError, subprocess.SubprocessError):
        pass
    return "unknown"


def make_workload(name: str):
    import synth
    if name == "c2":
        return synth.c2()
    if name == "c3":
        return synth.c3()
    if name == "c1":
        return synth.c1()
    if name == "c2p":
        return synth.c2()   # the same scene, run in paper mode
    raise SystemExit("unknown workload %r" % name)


def ablation_modes(d_features: int):
    """The ablation of Sec. 5.3's choices, as (name, Stream keyword arguments).

    Plain RLS (w = 1, Eq. 10) against weighted RLS, with the supplied
    features and with the paper's temporal feature (Eq. 12).  The prior
    P0 = I/delta acts like delta samples of unit weight (scaling every w by c
    equals scaling delta by 1/c), so delta is given in each mode's weight
    units: one unit-weight sample for w = 1 and for the Eq. 13 weight (at
    most 1), one median-weight sample (1 / median variance) for inverse
    variance weights.  A very large h makes the Eq. 13 weight 1 everywhere.
    The last mode adds the automatic forgetting factor (sigma0 60, lambda in
    [0.5, 0.98]) to weighted RLS."""
    import math
    import synth
    return [
        ("rls_features", dict(d=d_features, weight_mode="one", delta=1.0)),
        ("wrls_features", dict(d=d_features, weight_mode="invvar", delta=math.exp(-synth.VAR_MU))),
        ("rls_temporal_feature", dict(d=4, weight_mode="paper", h=1e3)),
        ("wrls_temporal_feature", dict(d=4, weight_mode="paper")),
        ("wrls_features_auto_lambda", dict(d=d_features, weight_mode="invvar",
                                           delta=math.exp(-synth.VAR_MU), sigma0=60.0, lam_min=0.5)),
    ]


def run_ablation(width: int, height: int, frames: int, warm: int, sigma_s: float = 1.5,
                 sigma_r: float = 0.15, sweep=(0.05, 0.15, 0.5, float("inf")), scene: str = "c2"):
    """PSNR (peak 1, linear) against the clean frames, over frames warm..end,
    of the temporal output and of the spatially blended output of every
    ablation mode, on the c2 scene (sub-pixel pan, disocclusions,
    heteroscedastic 1-spp noise) or the c3 scene (orbit, colour-LUT edit at
    frame 15, light change at 22; d = 10, FP16 inputs) at the given size;
    also the temporal flicker, the RMS frame-to-frame change of the error.
    Everything runs through libwrls on the GPU."""
    import math
    import torch
    import synth
    from paper_2106_08034_amd import wrls
    wl = (synth.c3 if scene == "c3" else synth.c2)(width=width, height=height, frames=frames)
    src = synth.FrameSource(wl)
    dev = torch.device("cuda:0")
    up = lambda a: torch.from_numpy(a).to(dev)
    seq = []
    for _ in range(frames):
        f = src.next()
        seq.append(tuple(up(a) for a in (f.color, f.feats, f.var, f.motion, f.clean)))

    def psnr(mse):
        return round(10.0 * math.log10(1.0 / mse), 3)

    res = {"input": {"psnr_db": psnr(float(sum(((c.float() - cl) ** 2).mean().item()
                                                   for c, _, _, _, cl in seq[warm:]) / (frames - warm)))}}
    for name, kw in ablation_modes(wl.d):
        d = kw.pop("d")
        paper = kw["weight_mode"] == "paper"
        st = wrls.Stream(width, height, d, in_dtype=wl.in_dtype, **kw)
        sigmas = [(sigma_s, sigma_r)] + ([(sigma_s, r) for r in sweep] if name == "wrls_features" else [])
        se_t, se_b = 0.0, [0.0] * len(sigmas)
        fl_t, fl_b, prev_t, prev_b = 0.0, 0.0, None, None
        for t, (c, fe, v, m, cl) in enumerate(seq):
            out = st.step(c, None if paper else fe, v if kw["weight_mode"] == "invvar" else None, m)
            blends = [st.blend(None if paper else fe, out, a, b) for a, b in sigmas]
            if t >= warm:
                e_t, e_b = out - cl, blends[0] - cl
                se_t += (e_t ** 2).mean().item()
                for i, bl in enumerate(blends):
                    se_b[i] += ((bl - cl) ** 2).mean().item()
                if prev_t is not None:
                    fl_t += ((e_t - prev_t) ** 2).mean().sqrt().item()
                    fl_b += ((e_b - prev_b) ** 2).mean().sqrt().item()
                prev_t, prev_b = e_t, e_b
        n = frames - warm
        rec = {"psnr_db": psnr(se_t / n), "psnr_blend_db": psnr(se_b[0] / n),
               "flicker": round(fl_t / (n - 1), 5), "flicker_blend": round(fl_b / (n - 1), 5),
               "stream": dict(kw, d=d)}
        if len(sigmas) > 1:
            rec["blend_sigma_r_sweep_db"] = {str(b): psnr(se_b[i] / n) for i, (_, b) in
                                             enumerate(sigmas) if i > 0}
        res[name] = rec
        st.close()
    return res


def _frame_pools(torch, shapes, count, host=None):
    """Device frames of the serving recipe, `count` per (width, height);
    host, if given, receives the host frames of the smallest 32-session
    trace resolution."""
    import synth
    pools = {}
    smallest = min(synth.C5_RESOLUTIONS, key=lambda s: s[0] * s[1])
    for i, (w, h) in enumerate(shapes):
        src = synth.FrameSource(synth.c5_frame_pool(w, h, count), stream=i)
        frames = [src.next() for _ in range(count)]
        if host is not None and (w, h) == smallest:
            host[(w, h)] = frames
        pools[(w, h)] = [tuple(torch.from_numpy(a).cuda() for a in (f.color, f.feats, f.var, f.motion))
                         for f in frames]
    torch.cuda.synchronize()
    return pools


def serving_parity(torch, session, recorded, host_frames):
    """G1 of a served session's outputs (host copies, in frame order) against
    the FP64 oracle fed the same cycled frames."""
    import oracle
    o = oracle.Oracle(session.width, session.height, 8, lam=0.98)
    par = _Parity(torch)
    for k, out in enumerate(recorded):
        f = host_frames[k % len(host_frames)]
        ref, scale = o.step(f.color, f.feats, f.var, f.motion, want_scale=True)
        par.add(out.cuda(), ref, scale)
    r = par.report()
    r["session"] = "%dx%d (sid %d), served batched" % (session.width, session.height, session.sid)
    return r


def bench_serving(args, modes=("batched", "per_stream"), saturating=True):
    """32 sessions (Poisson 4/s arrivals, Exp(20 s) durations, 720p..4K,
    30..60 Hz, FP16, d = 8) served in real time for args.serve_seconds:
    HBM-budget admission, continuous batching with two steps in flight, or
    the per-stream baseline (one launch per frame).  With `saturating`, the
    same sessions again at 16 arrivals/s and 120-240 Hz (more pixels per
    second than the GPU steps), also batched with admission by pixel rate,
    and at small resolutions and 240-480 Hz (launch-bound), each for
    args.saturating_seconds.  Returns {trace: {mode: report}} (Mpix/s,
    p50/p99 latency, ...) and the oracle check of one served session."""
    import torch

    import synth
    from paper_2106_08034_amd.serve import SATURATING, SMALL_FRAMES, Server

    t0 = time.time()
    host_pools = {}
    shapes = list(synth.C5_RESOLUTIONS) + [r for r in SMALL_FRAMES["resolutions"]
                                           if r not in synth.C5_RESOLUTIONS]
    pools = _frame_pools(torch, shapes, args.pool, host_pools)
    print("serving: generated %d frames per resolution in %.1fs" % (args.pool, time.time() - t0),
          file=sys.stderr, flush=True)
    budget = int((args.budget_gb or 200.0) * (1 << 30))
    traces = [("c5", synth.c5_sessions(), args.serve_seconds)]
    if saturating:
        traces.append(("c5_saturating", synth.c5_sessions(**SATURATING), args.saturating_seconds))
        traces.append(("small_frames", synth.c5_sessions(**SMALL_FRAMES), args.saturating_seconds))
    # rate-limited admission on the saturating trace: sessions wait for
    # admission instead of their frames queueing behind a backlog
    rate_budget = args.serve_rate_gpx * 1e9 if args.serve_rate_gpx > 0 else None
    out = {}
    # the served outputs of one session (the first of the smallest resolution
    # of the plain trace, its first 20 frames) are checked against the oracle
    # fed the same frames
    small = min(traces[0][1], key=lambda x: (x.width * x.height, x.sid))
    recorded = None
    for name, sessions, seconds in traces:
        out[name] = {}
        for mode in modes:
            srv = Server(budget_bytes=budget, max_batch=32, per_stream=mode == "per_stream",
                         tile=tuple(args.serve_tile))
            rec_sid = small.sid if (name == "c5" and mode == "batched") else None
            res, rec = srv.run(sessions, pools, seconds=seconds, record=rec_sid, record_frames=20,
                               poll=args.serve_poll_us * 1e-6)
            if rec_sid is not None:
                recorded = rec
            res["budget_gb"] = round(budget / (1 << 30), 2)
            res["frames_cycled_per_resolution"] = args.pool
            out[name][mode] = res
            print("serving %s %s: %.0f Mpix/s, p50 %.3f ms, p99 %.3f ms" % (
                name, mode, res["mpix_per_s"], res["p50_ms"], res["p99_ms"]), file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            srv.close()
            del srv
            gc.collect()
            torch.cuda.empty_cache()
        if name == "c5_saturating" and rate_budget is not None:
            for mode in modes:
                srv = Server(budget_bytes=budget, max_batch=32, tile=tuple(args.serve_tile),
                             rate_budget=rate_budget, per_stream=mode == "per_stream")
                res, _ = srv.run(sessions, pools, seconds=seconds, poll=args.serve_poll_us * 1e-6)
                res["budget_gb"] = round(budget / (1 << 30), 2)
                out[name + "_rate_admission"] = out.get(name + "_rate_admission", {})
                out[name + "_rate_admission"][mode] = res
                print("serving %s %s with rate admission: %.0f Mpix/s, p50 %.3f ms, p99 %.3f ms" % (
                    name, mode, res["mpix_per_s"], res["p50_ms"], res["p99_ms"]), file=sys.stderr,
                    flush=True)
                torch.cuda.synchronize()
                srv.close()
                del srv
                gc.collect()
                torch.cuda.empty_cache()
    if recorded:
        out["parity"] = serving_parity(torch, small, recorded, host_pools[(small.width, small.height)])
    if "batched" in modes and "per_stream" in modes:
        for name in out:
            if name == "parity":
                continue
            b, s = out[name]["batched"], out[name]["per_stream"]
            out[name]["batched_over_per_stream"] = {
                "mpix_per_s": round(b["mpix_per_s"] / max(s["mpix_per_s"], 1e-9), 3),
                "p99_ms": round(b["p99_ms"] / max(s["p99_ms"], 1e-9), 3)}
    return out


def bench_batched(args, tune: bool, small: bool = True):
    """16 streams of mixed resolution (640x480 .. 2560x1440), FP16 inputs,
    d = 8: one batched launch per round (HIP graph replay) against 16
    per-stream launches per round on the same HIP stream; with `small`, the
    same for 64 streams of 320x240, where launch overhead dominates."""
    import torch

    import synth
    from paper_2106_08034_amd import wrls

    wls = synth.c4_streams()
    t0 = time.time()
    pools, host_pools = [], []
    for wl in wls:
        src = synth.FrameSource(wl)
        frames = [src.next() for _ in range(args.pool)]
        host_pools.append(frames)
        pools.append([tuple(torch.from_numpy(a).cuda() for a in (f.color, f.feats, f.var, f.motion))
                      for f in frames])
    torch.cuda.synchronize()
    print("generated %d frames for %d streams in %.1fs" % (args.pool * len(wls), len(wls),
                                                          time.time() - t0), file=sys.stderr, flush=True)
    tune_ms = None
    if tune:
        from paper_2106_08034_amd import autotune
        shapes = [(wl.width, wl.height) for wl in wls]
        best, tune_ms = autotune.tune_batch(shapes, 8, pools, "f16", cache=autotune.TuneCache(None),
                                            force=True)
        print("autotuned batch launch shape %s" % (best,), file=sys.stderr, flush=True)
    else:
        best = tuple(args.batch_tile)
    batch = wrls.Batch(len(wls), 8, "f16")
    batch.set_tile(*best)
    hs = batch.hip_stream
    ext = torch.cuda.ExternalStream(hs)
    mixed = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=hs) for wl in wls]
    single = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=hs) for wl in wls]
    for s in single:  # the per-stream baseline gets the same tile
        s.set_tile(best[0], best[1], 0)
    outs = [torch.empty((3, wl.height, wl.width), device="cuda") for wl in wls]
    npix = sum(wl.width * wl.height for wl in wls)
    K, W = args.steps, args.warmup

    def round_batched(i):
        batch.step(mixed, [p[i % len(p)] for p in pools], outs)

    def round_single(i):
        for s, p, o in zip(single, pools, outs):
            s.step(*p[i % len(p)], out=o)

    res = {}
    for name, fn in (("batched_graph", round_batched), ("per_stream_launches", round_single)):
        with torch.cuda.stream(ext):
            for i in range(W):
                fn(i)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t_start = time.perf_counter()
            e0.record(ext)
            for i in range(K):
                fn(W + i)
            e1.record(ext)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t_start
        res[name] = {"ms_per_round": e0.elapsed_time(e1) / K, "wall_ms_per_round": wall * 1e3 / K}
    small_res = None
    if small:
        sm_wl = [synth.Workload(name="small-%02d" % i, width=320, height=240, frames=args.pool, d=8,
                                in_dtype="f16", motion="pan", pan=(2.3, 0.0), disocclusion=0.05,
                                config_index=3) for i in range(64)]
        spools = []
        for i, wl in enumerate(sm_wl):
            src = synth.FrameSource(wl, stream=i)
            spools.append([tuple(torch.from_numpy(a).cuda() for a in (f.color, f.feats, f.var, f.motion))
                           for f in (src.next() for _ in range(2))])
        sb = wrls.Batch(len(sm_wl), 8, "f16")
        sm = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=sb.hip_stream) for wl in sm_wl]
        ss = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=sb.hip_stream) for wl in sm_wl]
        souts = [torch.empty((3, wl.height, wl.width), device="cuda") for wl in sm_wl]
        sext = torch.cuda.ExternalStream(sb.hip_stream)
        small_res = {}
        for name, fn in (("batched_graph", lambda i: sb.step(sm, [p[i % 2] for p in spools], souts)),
                         ("per_stream_launches",
                          lambda i: [s.step(*p[i % 2], out=o) for s, p, o in zip(ss, spools, souts)])):
            with torch.cuda.stream(sext):
                for i in range(W):
                    fn(i)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(sext)
                for i in range(K):
                    fn(W + i)
                e1.record(sext)
                torch.cuda.synchronize()
            small_res[name] = round(e0.elapsed_time(e1) / K, 4)
        small_res["batched_speedup"] = round(small_res["per_stream_launches"] / small_res["batched_graph"], 3)
    # parity: fresh streams through the same batched launch over the pooled
    # frames, every stream against the FP64 oracle fed the same frames
    import oracle
    fresh = [wrls.Stream(wl.width, wl.height, 8, in_dtype="f16", hip_stream=hs) for wl in wls]
    gpu_outs = []
    with torch.cuda.stream(ext):
        for t in range(args.pool):
            o_t = [torch.empty((3, wl.height, wl.width), device="cuda") for wl in wls]
            batch.step(fresh, [p[t] for p in pools], o_t)
            gpu_outs.append(o_t)
    torch.cuda.synchronize()
    par = _Parity(torch)
    cpu_s = 0.0
    for i, wl in enumerate(wls):
        o = oracle.Oracle(wl.width, wl.height, 8, lam=0.98)
        for t in range(args.pool):
            f = host_pools[i][t]
            tc = time.perf_counter()
            ref, scale = o.step(f.color, f.feats, f.var, f.motion, want_scale=True)
            cpu_s += time.perf_counter() - tc
            par.add(gpu_outs[t][i], ref, scale)
        del o
    parity = par.report()
    parity["streams"] = len(wls)
    cpu = {"value": round(npix * args.pool / cpu_s / 1e6, 3), "unit": "Mpix/s", "cores": oracle.threads(),
           "cpu_model": cpu_model(), "kind": "oracle",
           "sample": "FP64 C oracle (OpenMP over rows), the first %d frames of each of the %d streams "
                     "(the parity pass, which also returns each output's term magnitude), %.1f s"
                     % (args.pool, len(wls), cpu_s)}
    del gpu_outs, fresh
    bpp = algorithmic_bytes_per_pixel(8, 2)
    b_ms = res["batched_graph"]["ms_per_round"]
    s_ms = res["per_stream_launches"]["ms_per_round"]
    gbs = bpp * npix / (b_ms / 1e3) / 1e9
    return {
        "workload": "c4-16-streams-mixed-640x480..2560x1440-d8-f16",
        "streams": len(wls), "pixels_per_round": npix,
        "resolutions": ["%dx%d" % (wl.width, wl.height) for wl in wls],
        "frames_cycled_per_stream": args.pool,
        "launch_shape": {"tile_w_log2": best[0], "block_threads": best[1], "blocks_per_cu": best[2],
                         "autotuned": tune,
                         "candidates_ms": ({k: round(v, 4) for k, v in tune_ms.items()}
                                           if tune_ms else None)},
        "batched": {"ms_per_round": round(b_ms, 4), "value": round(npix / (b_ms / 1e3) / 1e6, 2),
                    "unit": "Mpix/s",
                    "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                 "kernel": "wrls batch_kernel<8, f16>",
                                 "algorithmic_bytes_per_pixel": bpp}},
        "per_stream_launches": {"ms_per_round": round(s_ms, 4),
                                "value": round(npix / (s_ms / 1e3) / 1e6, 2), "unit": "Mpix/s"},
        "batched_speedup": round(s_ms / b_ms, 4),
        "wall_ms_per_round": {k: round(v["wall_ms_per_round"], 4) for k, v in res.items()},
        "small_frames_64x320x240_ms_per_round": small_res,
        "parity": parity,
        "cpu_baseline": cpu,
    }


class _Parity:
    """Running error of GPU outputs against the oracle's, per frame:
    G1 = max |gpu - ref| / max(|ref|, s, 1e-3 RMS(ref)) with s the magnitude
    of the output's terms (the parity tests' gate, 1e-4), and the error with
    |ref| alone as the denominator (floored at 1e-3 RMS).  Computed on the
    GPU in float64."""

    def __init__(self, torch):
        self.torch = torch
        self.g1 = 0.0
        self.y_rel = 0.0
        self.frames = 0

    def add(self, gpu_out, ref, scale):
        torch = self.torch
        r = torch.from_numpy(ref).cuda()
        g = gpu_out.double()
        tau = 1e-3 * float(torch.sqrt(torch.mean(r * r)))
        diff = (g - r).abs()
        den_y = torch.clamp(r.abs(), min=max(tau, 1e-30))
        self.y_rel = max(self.y_rel, float((diff / den_y).max()))
        if scale is not None:
            den = torch.maximum(den_y, torch.from_numpy(scale).cuda())
            self.g1 = max(self.g1, float((diff / den).max()))
        self.frames += 1

    def report(self):
        return {"frames": self.frames, "g1_max": float("%.3g" % self.g1),
                "y_relative_max": float("%.3g" % self.y_rel), "g1_bar": 1e-4,
                "within_bar": self.g1 <= 1e-4}


def bench_step(args, workload: str, with_cpu: bool, parity_frames=None, with_blend: bool = True):
    """One per-frame workload through wrls_step: K timed steps over the
    uploaded sequence, the roofline of the step kernel, the spatial blend,
    and (with_cpu) the oracle timed on the host over the same frames, whose
    outputs also give the parity of a GPU pass from frame 0; parity_frames
    limits that pass (None: all frames of the oracle sample)."""
    import numpy as np
    import torch

    import synth
    from paper_2106_08034_amd import wrls

    wl = make_workload(workload)
    paper = workload == "c2p"
    d_model = 4 if paper else wl.d
    dev = torch.device("cuda:0")
    t0 = time.time()
    src = synth.FrameSource(wl)
    host_frames, dev_frames = [], []
    n_unrounded = args.unrounded_frames if wl.in_dtype == "f16" else 0
    up = lambda a: torch.from_numpy(a).to(dev)
    for t in range(wl.frames):
        f = src.next(keep_unrounded=t < n_unrounded)
        host_frames.append(f)
        if paper:  # features and variance are not inputs of paper mode
            dev_frames.append((up(f.color), None, None, up(f.motion)))
        else:
            dev_frames.append(tuple(up(a) for a in (f.color, f.feats, f.var, f.motion)))
    torch.cuda.synchronize()
    print("generated and uploaded %d frames of %s in %.1fs" % (wl.frames, wl.name, time.time() - t0),
          file=sys.stderr, flush=True)

    stream = wrls.Stream(wl.width, wl.height, d_model, lam=0.98, in_dtype=wl.in_dtype,
                         weight_mode="paper" if paper else "invvar")
    out = torch.empty((3, wl.height, wl.width), dtype=torch.float32, device=dev)
    cs = torch.cuda.current_stream()
    for i in range(args.warmup):
        stream.step(*dev_frames[i % wl.frames], out=out)
    torch.cuda.synchronize()

    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record(cs)
    for i in range(K):
        stream.step(*dev_frames[(args.warmup + i) % wl.frames], out=out)
        ev[i + 1].record(cs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    per_launch_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(K)]
    total_ev_ms = ev[0].elapsed_time(ev[K])
    npix = wl.width * wl.height
    in_bytes = 2 if wl.in_dtype == "f16" else 4
    if paper:
        bpp = algorithmic_bytes_per_pixel_paper(in_bytes, motion=wl.motion != "static")
    else:
        bpp = algorithmic_bytes_per_pixel(wl.d, in_bytes, motion=wl.motion != "static")
    avg_launch_s = float(np.mean(per_launch_ms)) / 1e3
    achieved_gbs = bpp * npix / avg_launch_s / 1e9
    copy_gbs = measure_copy_gbs(torch, wrls, bpp * npix)
    res = {
        "value": round(K * npix / elapsed / 1e6, 2), "unit": "Mpix/s",
        "ms_per_step": round(elapsed * 1e3 / K, 4),
        "dtype": "f32" if wl.in_dtype == "f32" else "f32 (f16 inputs)",
        "config": {"workload": wl.name + ("-paper-mode-d4" if paper else ""),
                   "width": wl.width, "height": wl.height, "d": d_model,
                   "frames_in_sequence": wl.frames, "lambda": 0.98,
                   "input_dtype": wl.in_dtype, "state_dtype": "f32"},
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(workload),
                     "kernel": "wrls paper_step_kernel" if paper else "wrls step_kernel<%d>" % wl.d,
                     "algorithmic_bytes_per_pixel": bpp,
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "launch_us_min_max": [round(min(per_launch_ms) * 1e3, 2),
                                           round(max(per_launch_ms) * 1e3, 2)],
                     "event_total_ms": round(total_ev_ms, 3),
                     "measured_copy": {"kernel": "wrls_device_copy, same bytes per launch",
                                       "gbs": round(copy_gbs, 1),
                                       "frac": round(achieved_gbs / copy_gbs, 4)}},
    }
    probe_gbs = measure_probe_gbs(torch, stream, dev_frames, max(K, 10), bpp * npix)
    res["roofline"]["measured_probe"] = {
        "kernel": "wrls_traffic_probe: the step's loads and stores, same bytes per launch, "
                  "without reprojection or arithmetic",
        "gbs": round(probe_gbs, 1), "frac": round(achieved_gbs / probe_gbs, 4)}

    if with_blend:
        # the spatial blend (a second kernel after the step), timed on its
        # own over the last state: K launches, HIP events on the launch stream
        f_last = dev_frames[(args.warmup + K - 1) % wl.frames][1]
        fin = torch.empty_like(out)
        ss, sr = args.blend_sigmas
        stream.blend(f_last, out, ss, sr, out=fin)
        torch.cuda.synchronize()
        evb = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
        evb[0].record(cs)
        for i in range(K):
            stream.blend(f_last, out, ss, sr, out=fin)
            evb[i + 1].record(cs)
        torch.cuda.synchronize()
        blend_s = float(np.mean([evb[i].elapsed_time(evb[i + 1]) for i in range(K)])) / 1e3
        bbpp = blend_bytes_per_pixel(d_model, in_bytes, paper)
        bflop = blend_flop_per_pixel(d_model)
        alu_tflops = bflop * npix / blend_s / 1e12
        res["spatial_blend"] = {
            "kernel": "wrls blend_kernel<%d>" % d_model, "sigma_s": ss, "sigma_r": sr,
            "avg_launch_us": round(blend_s * 1e6, 2), "mpix_per_s": round(npix / blend_s / 1e6, 1),
            "algorithmic_bytes_per_pixel": bbpp,
            "achieved": round(bbpp * npix / blend_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(bbpp * npix / blend_s / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": load_traffic(workload, "blend"),
            "step_plus_blend_mpix_per_s": round(npix / (avg_launch_s + blend_s) / 1e6, 1),
            # the blend's arithmetic rate against the FP32 vector peak without
            # packed instructions (the build's), and the packed peak's fraction
            "alu": {"bound": "alu", "flop_per_pixel": bflop, "achieved": round(alu_tflops, 2),
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(alu_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                    "frac_of_packed_peak": round(alu_tflops / FP32_PACKED_PEAK_TFLOPS, 4)}}
    stream.close()

    if with_cpu or parity_frames:
        # The oracle as it stands on the same frames.  Its first pass also
        # gives the reference outputs of a GPU pass from frame 0 (a fresh
        # stream), compared frame by frame; further passes until about 10 s
        # of CPU work time it.
        import oracle
        n_cpu = args.cpu_frames or wl.frames
        n_par = n_cpu if parity_frames is None else min(parity_frames, n_cpu)

        def make_oracle():
            if paper:
                return oracle.Oracle(wl.width, wl.height, 4, lam=0.98, wmode=oracle.W_PAPER)
            return oracle.Oracle(wl.width, wl.height, wl.d, lam=0.98)

        def step_oracle(o, f, want_scale=False, unrounded=False):
            c = f.color_f32 if unrounded else f.color
            fe = f.feats_f32 if unrounded else f.feats
            if paper:
                return o.step(c, None, None, f.motion, want_scale=want_scale)
            return o.step(c, fe, f.var, f.motion, want_scale=want_scale)

        gpu = wrls.Stream(wl.width, wl.height, d_model, lam=0.98, in_dtype=wl.in_dtype,
                          weight_mode="paper" if paper else "invvar")
        par = _Parity(torch)
        par32 = _Parity(torch)
        o = make_oracle()
        o32 = make_oracle() if n_unrounded else None
        cpu_s = 0.0
        for t, f in enumerate(host_frames[:n_cpu] if with_cpu else host_frames[:n_par]):
            tc = time.perf_counter()
            r = step_oracle(o, f, want_scale=t < n_par)
            cpu_s += time.perf_counter() - tc
            if t < n_par:
                ref, scale = r
                g = gpu.step(*dev_frames[t])
                par.add(g, ref, scale)
                if o32 is not None and t < n_unrounded:
                    par32.add(g, *step_oracle(o32, f, want_scale=True, unrounded=True))
        del o, o32
        gpu.close()
        p = par.report()
        p["reference"] = "FP64 oracle on the same inputs (FP16-rounded where the workload is FP16)"
        if n_unrounded:
            p["vs_unrounded_fp32_inputs"] = {
                "frames": par32.frames, "g1_max": float("%.3g" % par32.g1),
                "y_relative_max": float("%.3g" % par32.y_rel),
                "note": "GPU on FP16 inputs against the oracle fed the unrounded FP32 inputs: "
                        "measures the binary16 rounding of colour and features"}
        res["parity"] = p
        if with_cpu:
            passes, frames_done = 1, n_cpu
            while passes < 8 and cpu_s < 10.0:
                o = make_oracle()
                tc = time.perf_counter()
                for f in host_frames[:n_cpu]:
                    step_oracle(o, f)
                cpu_s += time.perf_counter() - tc
                del o
                passes += 1
                frames_done += n_cpu
            cores = oracle.threads()
            cpu = {"value": round(frames_done * npix / cpu_s / 1e6, 3), "unit": "Mpix/s",
                   "cores": cores, "cpu_model": cpu_model(), "kind": "oracle",
                   "sample": "FP64 C oracle (OpenMP over rows), %d pass(es) over the first %d frames "
                             "of the same %s sequence, %.1f s (the first pass also returns each "
                             "output's term magnitude, the parity reference)" % (passes, n_cpu, wl.name,
                                                                                  cpu_s)}
            # the same oracle on one thread, over the first frame(s)
            oracle.set_threads(1)
            n1 = min(args.single_thread_frames, n_cpu)
            o = make_oracle()
            t1 = time.perf_counter()
            for f in host_frames[:n1]:
                step_oracle(o, f)
            s1 = time.perf_counter() - t1
            del o
            oracle.set_threads(cores)
            cpu["single_thread"] = {"value": round(n1 * npix / s1 / 1e6, 3), "unit": "Mpix/s",
                                    "sample": "the first %d frame(s), %.1f s" % (n1, s1)}
            res["cpu_baseline"] = cpu
    del dev_frames, host_frames
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3",
                    choices=["c1", "c2", "c2p", "c3", "c4", "c5", "ablation", "ablation_c3"],
                    help="c3 (default): the 4K d = 10 FP16 headline plus the c2, c4 and "
                         "serving legs; c2p: the c2 scene with the paper's own predictor and "
                         "weight (Eq. 12-13, d = 4); ablation: PSNR of RLS vs weighted RLS, "
                         "supplied vs temporal feature, fixed vs automatic lambda, with and "
                         "without the blend (ablation_c3: on the c3 scene with its edits)")
    ap.add_argument("--headline-only", action="store_true",
                    help="c3: skip the c2, c4 and serving legs")
    ap.add_argument("--serve-poll-us", type=float, default=0.0,
                    help="serving: host sleep between polls when nothing was launched (0: busy poll, "
                         "the default: a sleep costs the loop's latency its granularity)")
    ap.add_argument("--serve-seconds", type=float, default=12.0,
                    help="wall seconds of serving the 32-session trace, per mode")
    ap.add_argument("--saturating-seconds", type=float, default=8.0,
                    help="wall seconds of serving the saturating trace, per mode")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="serving: HBM budget for session state (0: 200 GB)")
    ap.add_argument("--serve-rate-gpx", type=float, default=8.0,
                    help="saturating trace: also serve it batched with admission limited to this "
                         "many Gpx/s offered (0: skip)")
    ap.add_argument("--pool", type=int, default=0,
                    help="distinct frames generated per stream (c4) or per resolution "
                         "(serving), cycled (0: 4 in the default run, 60 with --workload c5)")
    ap.add_argument("--tune", action="store_true", help="c4: autotune the batched launch shape")
    ap.add_argument("--batch-tile", type=int, nargs=3, default=(8, 256, 0),
                    metavar=("TILE_W_LOG2", "BLOCK_THREADS", "BLOCKS_PER_CU"),
                    help="c4 launch shape without --tune (default: 256 x 1 tiles, one workgroup "
                         "per tile, the autotuner's pick on the c4 mix)")
    ap.add_argument("--serve-tile", type=int, nargs=3, default=(8, 256, 0),
                    metavar=("TILE_W_LOG2", "BLOCK_THREADS", "BLOCKS_PER_CU"),
                    help="serving launch shape (both modes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--blend-sigmas", type=float, nargs=2, default=(1.5, 0.15),
                    metavar=("SIGMA_S", "SIGMA_R"),
                    help="widths of the timed 5x5 spatial blend (after the step loop)")
    ap.add_argument("--cpu-frames", type=int, default=0,
                    help="frames of the oracle sample (0: all frames of the sequence)")
    ap.add_argument("--single-thread-frames", type=int, default=1,
                    help="frames of the one-thread oracle sample")
    ap.add_argument("--unrounded-frames", type=int, default=6,
                    help="FP16 workloads: frames compared against the oracle fed the unrounded "
                         "FP32 inputs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 10 plain device copies of MIB MiB (the known-size "
                         "reference for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copied 10 x %d MiB" % args.copy_calibration, flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: it measures one GPU's share of the work "
              "(a stream or an image band per GPU needs no collective); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2106_08034_amd import build as hip_build

    if hip_build.needs_build():
        hip_build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(torch.device("cuda:0"))
    base = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "data": DATA}

    if args.workload == "c4":
        args.pool = args.pool or 4
        r = bench_batched(args, tune=args.tune)
        line = dict(base, metric="denoised Mpix/s (wRLS step, batched) + % HBM roofline",
                    value=r["batched"]["value"], unit="Mpix/s",
                    ms_per_step=r["batched"]["ms_per_round"], dtype="f32 (f16 inputs)",
                    config={"workload": r["workload"]}, roofline=dict(r["batched"]["roofline"],
                                                                      traffic=None),
                    c4=r, cpu_baseline=r["cpu_baseline"])
        print(json.dumps(line), flush=True)
        return
    if args.workload in ("ablation", "ablation_c3"):
        c3 = args.workload == "ablation_c3"
        W, H = 640, 360
        T, warm = (30, 5) if c3 else (60, 10)
        t0 = time.perf_counter()
        res = run_ablation(W, H, T, warm, scene="c3" if c3 else "c2")
        best = max(v.get("psnr_blend_db", 0.0) for k, v in res.items() if k != "input")
        line = dict(base, metric="PSNR dB vs clean frames (ablation of Sec. 5.3)", value=best,
                    unit="dB", steps=T, warmup=warm,
                    ms_per_step=round((time.perf_counter() - t0) * 1e3 / T, 3), dtype="f32",
                    data="synthetic (seeded procedural scene with its clean frames)",
                    config={"workload": "%s-scene-%dx%d-%dframes-ablation" % ("c3" if c3 else "c2",
                                                                              W, H, T),
                            "psnr_frames": "%d..%d" % (warm, T - 1), "blend_sigmas": [1.5, 0.15]},
                    ablation=res, cpu_baseline=None)
        print(json.dumps(line), flush=True)
        return
    if args.workload == "c5":
        args.pool = args.pool or 60
        sv = bench_serving(args)
        b = sv["c5"]["batched"]
        line = dict(base, metric="denoised Mpix/s + p50/p99 frame latency @32 sessions (serving)",
                    value=b["mpix_per_s"], unit="Mpix/s", steps=b["steps"], warmup=0,
                    ms_per_step=round(b["seconds"] * 1e3 / max(1, b["steps"]), 4),
                    dtype="f32 (f16 inputs)", data="synthetic (seeded sessions and procedural frames)",
                    config={"workload": "c5-32-sessions-poisson4-exp20s-720p..4k-30..60Hz-d8-f16",
                            "serve_seconds": args.serve_seconds}, serving=sv, cpu_baseline=None)
        print(json.dumps(line), flush=True)
        return

    r = bench_step(args, args.workload, with_cpu=not args.no_cpu_baseline)
    line = dict(base, metric=METRIC if args.workload == "c3" else
                "denoised Mpix/s (wRLS step) + % HBM roofline", **r)
    line.setdefault("cpu_baseline", None)
    if args.workload == "c3" and not args.headline_only:
        # the other configurations, each in its own key
        c2 = bench_step(args, "c2", with_cpu=False, parity_frames=10, with_blend=True)
        line["c2"] = {k: c2[k] for k in ("value", "unit", "ms_per_step", "config", "roofline",
                                         "parity", "spatial_blend")}
        args.pool = args.pool or 4
        line["c4_batched"] = bench_batched(args, tune=args.tune)
        torch.cuda.empty_cache()
        line["serving"] = bench_serving(args)
        line["paper_context"] = bench_paper_context(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
