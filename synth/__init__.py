"""Seeded synthetic workloads for the wRLS temporal denoiser.

This module only draws inputs: a procedural scene standing in for the
paper's volume-rendered sequences (the volumes of its Table 3 and its
1024-spp references are not available), observed through heteroscedastic
1-spp-like noise, with the motion fields of a camera pan or a camera orbit.
It holds none of the denoiser's arithmetic; both the GPU path and the FP64
oracle consume exactly the arrays it returns.

Scene (normalised coordinates u = x / H, v = y / H, so the image content has
the same shape at every resolution):
  depth D in [0.2, 1): 0.2 plus six seeded Gaussian bumps;
  normal n = normalise(-dD/du, -dD/dv, 1);
  albedo in [0.05, 0.95]: smooth seeded sinusoids plus three hard edges
    (half-planes on seeded lines, each adding a seeded colour jump);
  clean colour = albedo * (0.2 + max(0, n . l)) for a seeded light l;
  two smooth "scattering depth" fields for the d = 10 predictor.
Observation per frame: every feature channel gets N(0, 0.1^2) noise; the
per-pixel variance is LogNormal(mu=-3, sigma=1) redrawn every frame; the
noisy colour is clean + sqrt(var) * N(0, 1) per channel (one sample per
pixel, unclamped, linear HDR).  FP16 workloads round colour and features to
binary16 (round to nearest even); variance and motion stay FP32.

Seeding: NumPy PCG64 with SeedSequence(210608034 + config index); the scene
of stream s comes from spawn_key (s, 0xC0FFEE), the noise of frame t in the
band of rows starting at r0 from spawn_key (s, t + 1, r0), and the
disocclusion discs of frame t from spawn_key (s, t + 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, Optional, Tuple

import numpy as np

SEED_BASE = 210608034
FEATURE_NOISE = 0.1
VAR_MU, VAR_SIGMA = -3.0, 1.0


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and structure of one synthetic sequence."""
    name: str
    width: int
    height: int
    frames: int
    d: int                      # predictor length, intercept included
    in_dtype: str               # "f32" or "f16" for colour and features
    motion: str                 # "static", "pan" or "orbit"
    pan: Tuple[float, float] = (0.0, 0.0)   # backward motion, pixels/frame
    disocclusion: float = 0.0   # fraction of pixels with NaN motion per frame
    orbit_deg: float = 0.0      # camera orbit per frame (degrees)
    lut_frame: Optional[int] = None    # transfer-function edit from this frame
    light_frame: Optional[int] = None  # light rotation from this frame
    config_index: int = 0       # seeds SeedSequence(SEED_BASE + config_index)

    @property
    def pixels(self) -> int:
        return self.width * self.height

    @property
    def np_in_dtype(self):
        return np.float16 if self.in_dtype == "f16" else np.float32


# The five workloads: the 64x64 static correctness case, the 1080p sub-pixel
# pan, the 4K orbit with appearance edits, the 16-stream batch and the
# 32-session serving mix.
def c1(**kw) -> Workload:
    base = dict(name="c1-64x64-static-d8-f32", width=64, height=64, frames=8, d=8,
                in_dtype="f32", motion="static", config_index=0)
    base.update(kw)
    return Workload(**base)


def c2(**kw) -> Workload:
    base = dict(name="c2-1920x1080-pan-d8-f32", width=1920, height=1080, frames=60, d=8,
                in_dtype="f32", motion="pan", pan=(2.3, 0.0), disocclusion=0.05,
                config_index=1)
    base.update(kw)
    return Workload(**base)


def c3(**kw) -> Workload:
    base = dict(name="c3-3840x2160-orbit-d10-f16", width=3840, height=2160, frames=30, d=10,
                in_dtype="f16", motion="orbit", orbit_deg=0.05, lut_frame=15, light_frame=22,
                config_index=2)
    base.update(kw)
    return Workload(**base)


C4_RESOLUTIONS = ((640, 480), (1280, 720), (1920, 1080), (2560, 1440))
C5_RESOLUTIONS = ((1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))


def c4_streams(n_streams: int = 16, frames: int = 120, scale: float = 1.0):
    """The batched workload: n_streams pans of seeded resolution and seeded
    direction (2.3 px/frame), FP16 inputs, d = 8.  `scale` shrinks every
    resolution (for parity tests at small sizes)."""
    ss = np.random.SeedSequence(SEED_BASE + 3)
    rng = np.random.Generator(np.random.PCG64(ss))
    out = []
    for s in range(n_streams):
        w, h = C4_RESOLUTIONS[int(rng.integers(len(C4_RESOLUTIONS)))]
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        w, h = max(8, int(round(w * scale))), max(8, int(round(h * scale)))
        out.append(Workload(name="c4-s%02d-%dx%d" % (s, w, h), width=w, height=h,
                            frames=frames, d=8, in_dtype="f16", motion="pan",
                            pan=(2.3 * math.cos(ang), 2.3 * math.sin(ang)),
                            disocclusion=0.05, config_index=3))
    return out


@dataclasses.dataclass
class Frame:
    color: np.ndarray    # (3, H, W) in_dtype
    feats: np.ndarray    # (d-1, H, W) in_dtype
    var: np.ndarray      # (H, W) float32
    motion: np.ndarray   # (2, H, W) float32, NaN = disoccluded
    clean: np.ndarray    # (3, H, W) float32, the noise-free colour
    color_f32: Optional[np.ndarray] = None  # colour before FP16 rounding (on request)
    feats_f32: Optional[np.ndarray] = None  # features before FP16 rounding (on request)


# Frames are generated in bands of rows, each with its own seeded noise, in a
# thread pool (NumPy releases the GIL inside its array kernels).
BAND_ROWS = 32
_POOL = None


def _pool():
    global _POOL
    if _POOL is None:
        import concurrent.futures
        import os
        n = min(16, os.cpu_count() or 1)
        _POOL = concurrent.futures.ThreadPoolExecutor(max_workers=n) if n > 1 else False
    return _POOL or None


class _Scene:
    """Seeded procedural scene evaluated analytically at (u, v)."""

    def __init__(self, rng: np.random.Generator, u_span: float):
        lo, hi = -0.1, u_span + 0.1
        self.bumps = [(rng.uniform(0.04, 0.13), rng.uniform(lo, hi), rng.uniform(-0.1, 1.1),
                       rng.uniform(0.08, 0.3)) for _ in range(6)]
        self.alb = [(rng.uniform(0.5, 3.0), rng.uniform(0, 1), rng.uniform(0.5, 3.0),
                     rng.uniform(0, 1), rng.uniform(1.0, 4.0), rng.uniform(0, 1))
                    for _ in range(3)]
        self.edges = []
        for _ in range(3):
            th = rng.uniform(0, 2 * math.pi)
            self.edges.append((math.cos(th), math.sin(th), rng.uniform(0.2 * u_span, 0.8 * u_span),
                               rng.uniform(0.2, 0.8), rng.uniform(-0.3, 0.3, size=3)))
        self.scatter = [(rng.uniform(0.5, 2.5), rng.uniform(0, 1), rng.uniform(0.5, 2.5),
                         rng.uniform(0, 1)) for _ in range(2)]
        l = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), 1.0])
        self.light = l / np.linalg.norm(l)
        knots_y = np.cumsum(rng.uniform(0.2, 1.0, size=(3, 8)), axis=1)
        self.lut_x = np.linspace(0.0, 1.25, 8)
        self.lut_y = 1.25 * (knots_y - knots_y[:, :1]) / (knots_y[:, -1:] - knots_y[:, :1])
        self.lut_y = self.lut_y[:, rng.permutation(8)] * 0.5 + self.lut_y * 0.5

    def depth_and_grad(self, u, v):
        D = 0.2
        gu = 0.0
        gv = 0.0
        for a, cu, cv, s in self.bumps:
            eu = np.exp(-((u - cu) ** 2) / (2 * s * s))
            ev = np.exp(-((v - cv) ** 2) / (2 * s * s))
            g = a * eu * ev
            D = D + g
            gu = gu - g * (u - cu) / (s * s)
            gv = gv - g * (v - cv) / (s * s)
        return D, gu, gv

    def albedo(self, u, v):
        chans = []
        for k1, p1, k2, p2, k3, p3 in self.alb:
            a = 0.5 + 0.2 * np.sin(2 * math.pi * (k1 * u + p1)) * np.cos(2 * math.pi * (k2 * v + p2))
            # sin(k3 (u + v) + p3), expanded so (1,W) x (H,1) grids stay separable
            su, cu = np.sin(2 * math.pi * (k3 * u + p3)), np.cos(2 * math.pi * (k3 * u + p3))
            sv, cv = np.sin(2 * math.pi * k3 * v), np.cos(2 * math.pi * k3 * v)
            chans.append(a + 0.1 * (su * cv + cu * sv))
        for cth, sth, pu, pv, jump in self.edges:
            side = ((u - pu) * cth + (v - pv) * sth) > 0
            for c in range(3):
                chans[c] = chans[c] + jump[c] * side
        return [np.clip(ch, 0.05, 0.95) for ch in chans]

    def scatter_fields(self, u, v):
        return [0.5 + 0.4 * np.sin(2 * math.pi * (k1 * u + p1)) * np.cos(2 * math.pi * (k2 * v + p2))
                for k1, p1, k2, p2 in self.scatter]


class FrameSource:
    """Frames of one workload, generated in order (the orbit chain needs the
    previous frame's scene coordinates)."""

    def __init__(self, wl: Workload, stream: int = 0):
        self.wl = wl
        self.stream = stream
        self.entropy = SEED_BASE + wl.config_index
        rng = self._rng(0xC0FFEE)
        W, H = wl.width, wl.height
        pan_extent = abs(wl.pan[0]) * wl.frames + abs(wl.pan[1]) * wl.frames
        self.scene = _Scene(rng, (W + pan_extent) / H)
        self.t = 0
        self._X = None  # orbit: scene pixel coordinates of every pixel
        if wl.motion == "orbit":
            self._orbit_flow = self._make_orbit_flow()

    def _rng(self, t: int) -> np.random.Generator:
        return np.random.Generator(np.random.PCG64(
            np.random.SeedSequence(self.entropy, spawn_key=(self.stream, t))))

    def _make_orbit_flow(self):
        """Backward flow of a pinhole camera (60 deg horizontal FOV) orbiting
        a pivot at depth 0.6 about the vertical axis, from the static depth
        map of the scene at its initial position."""
        wl = self.wl
        W, H = wl.width, wl.height
        x = np.arange(W, dtype=np.float64)[None, :]
        y = np.arange(H, dtype=np.float64)[:, None]
        D, _, _ = self.scene.depth_and_grad(x / H, y / H)
        f = (W / 2.0) / math.tan(math.radians(30.0))
        cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
        X = (x - cx) / f * D
        Y = (y - cy) / f * D + 0 * x
        Z = D + 0 * x
        th = -math.radians(wl.orbit_deg)
        pz = 0.6
        Xr = math.cos(th) * X + math.sin(th) * (Z - pz)
        Zr = -math.sin(th) * X + math.cos(th) * (Z - pz) + pz
        xp = cx + f * Xr / Zr
        yp = cy + f * Y / Zr
        return np.stack([xp - x, yp - y]).astype(np.float32)

    def _orbit_coords(self):
        """Scene pixel coordinates of every pixel at the current frame:
        X_t(x) = X_{t-1}(x + v(x)), sampled bilinearly and extended linearly
        outside the image."""
        wl = self.wl
        W, H = wl.width, wl.height
        if self._X is None:
            xs = np.broadcast_to(np.arange(W, dtype=np.float64)[None, :], (H, W))
            ys = np.broadcast_to(np.arange(H, dtype=np.float64)[:, None], (H, W))
            self._X = np.stack([xs, ys]).copy()
            return self._X
        prev = self._X
        new = np.empty_like(prev)

        def band(b):
            r0, r1 = b
            v = self._orbit_flow[:, r0:r1].astype(np.float64)
            sx = np.arange(W)[None, :] + v[0]
            sy = np.arange(r0, r1)[:, None] + v[1]
            cxs = np.clip(sx, 0, W - 1)
            cys = np.clip(sy, 0, H - 1)
            x0 = np.minimum(np.floor(cxs).astype(np.int64), W - 2 if W > 1 else 0)
            y0 = np.minimum(np.floor(cys).astype(np.int64), H - 2 if H > 1 else 0)
            fx, fy = cxs - x0, cys - y0
            x1, y1 = np.minimum(x0 + 1, W - 1), np.minimum(y0 + 1, H - 1)
            for c in range(2):
                P = prev[c]
                top = P[y0, x0] * (1 - fx) + P[y0, x1] * fx
                bot = P[y1, x0] * (1 - fx) + P[y1, x1] * fx
                new[c, r0:r1] = top * (1 - fy) + bot * fy
            new[0, r0:r1] += sx - cxs
            new[1, r0:r1] += sy - cys

        bands = [(r0, min(H, r0 + BAND_ROWS)) for r0 in range(0, H, BAND_ROWS)]
        pool = _pool()
        if pool is None:
            for b in bands:
                band(b)
        else:
            list(pool.map(band, bands))
        self._X = new
        return new

    def _disocclusion_mask(self, rng, W, H):
        frac = self.wl.disocclusion
        mask = np.zeros((H, W), dtype=bool)
        if frac <= 0:
            return mask
        r = max(2.0, 0.04 * H)
        n = max(1, int(round(frac * W * H / (math.pi * r * r))))
        cx = rng.uniform(0, W, size=n)
        cy = rng.uniform(0, H, size=n)
        for i in range(n):
            x0, x1 = max(0, int(cx[i] - r)), min(W, int(cx[i] + r) + 1)
            y0, y1 = max(0, int(cy[i] - r)), min(H, int(cy[i] + r) + 1)
            if x0 >= x1 or y0 >= y1:
                continue
            xx = np.arange(x0, x1)[None, :]
            yy = np.arange(y0, y1)[:, None]
            mask[y0:y1, x0:x1] |= (xx - cx[i]) ** 2 + (yy - cy[i]) ** 2 <= r * r
        return mask

    def _band(self, t, r0, r1, u, v, l, out):
        """Scene and noise of rows [r0, r1): fills the frame arrays in `out`.
        Each band draws its noise from its own seeded generator, so the
        result does not depend on how bands are scheduled."""
        wl = self.wl
        W = wl.width
        h = r1 - r0
        sc = self.scene
        rng = np.random.Generator(np.random.PCG64(
            np.random.SeedSequence(self.entropy, spawn_key=(self.stream, t + 1, r0))))
        D, gu, gv = sc.depth_and_grad(u, v)
        D = np.broadcast_to(D, (h, W))
        nrm = np.sqrt(gu * gu + gv * gv + 1.0)
        n = [np.broadcast_to(-gu / nrm, (h, W)), np.broadcast_to(-gv / nrm, (h, W)),
             np.broadcast_to(1.0 / nrm, (h, W))]
        alb = [np.broadcast_to(a, (h, W)) for a in sc.albedo(u, v)]
        shade = 0.2 + np.maximum(0.0, n[0] * l[0] + n[1] * l[1] + n[2] * l[2])
        clean = out["clean"][:, r0:r1]
        for c in range(3):
            clean[c] = alb[c] * shade
            if wl.lut_frame is not None and t >= wl.lut_frame:
                clean[c] = np.interp(clean[c], sc.lut_x, sc.lut_y[c])
        feats_clean = alb + n + [D]
        if wl.d == 10:
            feats_clean += [np.broadcast_to(s_, (h, W)) for s_ in sc.scatter_fields(u, v)]
        feats = out["feats32"][:, r0:r1]
        for i, fc in enumerate(feats_clean):
            feats[i] = fc + FEATURE_NOISE * rng.standard_normal((h, W), dtype=np.float32)
        var = np.exp(VAR_MU + VAR_SIGMA * rng.standard_normal((h, W), dtype=np.float32))
        out["var"][r0:r1] = var
        out["color32"][:, r0:r1] = clean + np.sqrt(var)[None] * rng.standard_normal((3, h, W), dtype=np.float32)

    def next(self, keep_unrounded: bool = False) -> Frame:
        wl = self.wl
        W, H, t = wl.width, wl.height, self.t
        if wl.d not in (8, 10):
            raise ValueError("the procedural scene provides d = 8 or d = 10 predictors")
        if wl.motion == "orbit":
            X = self._orbit_coords()
            U, V = (X[0] / H).astype(np.float32), (X[1] / H).astype(np.float32)
            motion = self._orbit_flow.copy()
        else:
            # content at frame t is the scene shifted by t * (-pan), so the
            # previous frame holds pixel x's content at x + pan
            U = ((np.arange(W, dtype=np.float64)[None, :] + wl.pan[0] * t) / H).astype(np.float32)
            V = ((np.arange(H, dtype=np.float64)[:, None] + wl.pan[1] * t) / H).astype(np.float32)
            motion = np.empty((2, H, W), np.float32)
            motion[0] = wl.pan[0]
            motion[1] = wl.pan[1]
        l = self.scene.light
        if wl.light_frame is not None and t >= wl.light_frame:
            th = math.radians(60.0)
            l = np.array([math.cos(th) * l[0] + math.sin(th) * l[2], l[1],
                          -math.sin(th) * l[0] + math.cos(th) * l[2]])
        l = [float(c) for c in l]
        out = {"clean": np.empty((3, H, W), np.float32),
               "feats32": np.empty((wl.d - 1, H, W), np.float32),
               "var": np.empty((H, W), np.float32),
               "color32": np.empty((3, H, W), np.float32)}
        bands = [(r0, min(H, r0 + BAND_ROWS)) for r0 in range(0, H, BAND_ROWS)]

        def work(b):
            r0, r1 = b
            if U.shape[0] == 1:
                u = U
            else:
                u = U[r0:r1]
            v = V[r0:r1]
            self._band(t, r0, r1, u, v, l, out)

        pool = _pool()
        if pool is None or len(bands) == 1:
            for b in bands:
                work(b)
        else:
            list(pool.map(work, bands))
        if wl.disocclusion > 0:
            rng = self._rng(t + 1)
            mask = self._disocclusion_mask(rng, W, H)
            motion[:, mask] = np.nan
        dt = wl.np_in_dtype
        self.t += 1
        fr = Frame(color=out["color32"].astype(dt), feats=out["feats32"].astype(dt), var=out["var"],
                   motion=motion, clean=out["clean"])
        if keep_unrounded:
            fr.color_f32, fr.feats_f32 = out["color32"], out["feats32"]
        return fr

    def __iter__(self) -> Iterator[Frame]:
        while self.t < self.wl.frames:
            yield self.next()


def frames(wl: Workload, stream: int = 0, count: Optional[int] = None):
    """The first `count` (default: all) frames of a workload, as a list."""
    src = FrameSource(wl, stream)
    n = wl.frames if count is None else count
    return [src.next() for _ in range(n)]


@dataclasses.dataclass(frozen=True)
class Session:
    """One viewer of the serving workload."""
    sid: int
    width: int
    height: int
    fps: float
    arrival: float    # seconds after the start
    duration: float   # seconds


def c5_sessions(n: int = 32, rate: float = 4.0, mean_duration: float = 20.0,
                resolutions=C5_RESOLUTIONS, fps_range=(30.0, 60.0)):
    """The serving workload: n sessions with Poisson(rate) arrivals,
    Exp(mean_duration) durations, a resolution drawn uniformly from
    `resolutions` and a frame rate uniform in fps_range."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + 4)))
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        out.append(Session(sid=i, width=w, height=h, fps=float(rng.uniform(*fps_range)),
                           arrival=float(arrivals[i]),
                           duration=float(rng.exponential(mean_duration))))
    return out


def c5_frame_pool(width: int, height: int, count: int, stream: int = 0) -> Workload:
    """Pre-generated frames of one serving resolution (pan, FP16, d = 8),
    cycled by the sessions of that resolution."""
    return Workload(name="c5-pool-%dx%d" % (width, height), width=width, height=height,
                    frames=count, d=8, in_dtype="f16", motion="pan", pan=(2.3, 0.0),
                    disocclusion=0.05, config_index=4)
