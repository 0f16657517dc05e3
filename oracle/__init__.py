"""FP64 CPU oracle of the per-pixel wRLS temporal denoiser (paper Sec. 5).

TEST INFRASTRUCTURE ONLY.  This package is the reference that the GPU
library is checked against: the C source ``wrls_oracle.c`` holds the
arithmetic (FP64, one pixel at a time, in the order of Eq. 8, 14, 9, 11 and
6); this module only marshals NumPy arrays into it.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wrls_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

W_INVVAR = 0
W_ONE = 1
W_PAPER = 2
INTERP_BILINEAR = 0
INTERP_NEAREST = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (binary64, no fast-math, no FMA
    contraction, OpenMP over image rows)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # A planted-mistake build of this oracle (see tests/test_oracle_mutants.py)
    # is loaded in place of the real one when this variable names it.
    path = os.environ.get("WRLS_ORACLE_LIB_OVERRIDE")
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_create.restype = ctypes.c_void_p
    lib.oracle_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.oracle_destroy.argtypes = [ctypes.c_void_p]
    lib.oracle_reset.argtypes = [ctypes.c_void_p]
    lib.oracle_frames.restype = ctypes.c_long
    lib.oracle_frames.argtypes = [ctypes.c_void_p]
    lib.oracle_set_paper_params.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double]
    lib.oracle_get_history.argtypes = [ctypes.c_void_p, dp]
    lib.oracle_set_history.argtypes = [ctypes.c_void_p, dp]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_step.restype = ctypes.c_int
    lib.oracle_step.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp, dp, dp, dp,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_set_forgetting.restype = ctypes.c_int
    lib.oracle_set_forgetting.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    lib.oracle_get_state.argtypes = [ctypes.c_void_p, dp, dp]
    lib.oracle_get_beta.argtypes = [ctypes.c_void_p, dp]
    lib.oracle_set_state.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_long]
    lib.oracle_blend.restype = ctypes.c_int
    lib.oracle_blend.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_double, dp]
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP threads the oracle's per-row loop uses."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Sets the OpenMP threads of the oracle's per-row loops."""
    _load().oracle_set_threads(int(n))


def _f64(a, shape):
    """Widen to a C-contiguous float64 array of the given shape (exact for
    float16 and float32 inputs)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One denoised image sequence held in FP64.

    lam: forgetting factor; delta: prior precision (P starts at I/delta,
    beta at 0); var_floor: smallest variance turned into a weight.
    sigma0 > 0: automatic forgetting factor (Fortescue, Kershenbaum and
    Ydstie): per pixel and step, lambda keeps the weighted a-posteriori
    error information at sigma0, limited to [lam_min, lam].
    wmode W_PAPER (d = 4): the predictor is the temporal feature of Eq. 12
    (alpha) and the weight that of Eq. 13 (h_bw, eps); features and variance
    are then not used.
    """

    def __init__(self, width, height, d, lam=0.98, delta=1.0, var_floor=1e-6,
                 wmode=W_INVVAR, interp=INTERP_BILINEAR, alpha=0.75, h_bw=0.75, eps=1e-4,
                 sigma0=0.0, lam_min=None):
        self._lib = _load()
        self.W, self.H, self.d = int(width), int(height), int(d)
        self.lam, self.delta = float(lam), float(delta)
        h = self._lib.oracle_create(self.W, self.H, self.d, self.lam, self.delta,
                                    float(var_floor), int(wmode), int(interp))
        if not h:
            raise ValueError("oracle_create rejected the parameters")
        self._h = h
        # paper mode (Eq. 12-13): history weight alpha, bandwidth h, epsilon
        self._lib.oracle_set_paper_params(h, float(alpha), float(h_bw), float(eps))
        lo = self.lam if lam_min is None else float(lam_min)
        if self._lib.oracle_set_forgetting(h, float(sigma0), lo) != 0:
            raise ValueError("oracle_set_forgetting rejected sigma0=%r, lam_min=%r" % (sigma0, lam_min))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_destroy(h)
            self._h = None

    @property
    def frames(self) -> int:
        return int(self._lib.oracle_frames(self._h))

    def reset(self):
        self._lib.oracle_reset(self._h)

    def step(self, color, feats, var, motion=None, roi=None, want_prior=False,
             want_lambda=False, want_scale=False):
        """Denoise one frame.  color (3,H,W); feats (d-1,H,W) or None when
        d = 1; var (H,W) or None; motion (2,H,W) or None (= zero).
        roi = (x0, y0, x1, y1) restricts the computed pixels.  Returns the
        a-posteriori prediction (3,H,W) float64; with any want_* flag, a
        tuple of it and, in this order, the a-priori prediction (3,H,W), the
        forgetting factor of each pixel (H,W), and the magnitude of the
        output's terms sum_i |p_i beta_c,i| (3,H,W) that were asked for."""
        W, H, d = self.W, self.H, self.d
        c = _f64(color, (3, H, W))
        f = _f64(feats, (d - 1, H, W)) if (d > 1 and feats is not None) else None
        v = _f64(var, (H, W)) if var is not None else None
        m = _f64(motion, (2, H, W)) if motion is not None else None
        out = np.zeros((3, H, W), np.float64)
        prior = np.zeros((3, H, W), np.float64) if want_prior else None
        lam = np.zeros((H, W), np.float64) if want_lambda else None
        scale = np.zeros((3, H, W), np.float64) if want_scale else None
        x0, y0, x1, y1 = roi if roi is not None else (0, 0, W, H)
        rc = self._lib.oracle_step(self._h, _ptr(c), _ptr(f), _ptr(v), _ptr(m), _ptr(out),
                                   _ptr(prior), _ptr(lam), _ptr(scale),
                                   int(x0), int(y0), int(x1), int(y1))
        if rc != 0:
            raise ValueError("oracle_step rejected the region %r" % (roi,))
        extra = [a for a, want in ((prior, want_prior), (lam, want_lambda), (scale, want_scale)) if want]
        return tuple([out] + extra) if extra else out

    def blend(self, feats, sigma_s, sigma_r):
        """The 5x5 spatial blend of neighbour-model predictions (Sec. 5.3) on
        the current state: feats (d-1,H,W) of the frame just stepped (None
        in paper mode); sigma_s in pixels, sigma_r in colour units (+inf
        turns a factor off).  Returns (3,H,W) float64."""
        W, H, d = self.W, self.H, self.d
        f = _f64(feats, (d - 1, H, W)) if (d > 1 and feats is not None) else None
        out = np.zeros((3, H, W), np.float64)
        rc = self._lib.oracle_blend(self._h, _ptr(f), float(sigma_s), float(sigma_r), _ptr(out))
        if rc != 0:
            raise ValueError("oracle_blend: no state yet, or features missing")
        return out

    def get_state(self):
        """(P, beta): P (d,d,H,W) full matrices, beta (3,d,H,W)."""
        W, H, d = self.W, self.H, self.d
        P = np.zeros((d, d, H, W), np.float64)
        beta = np.zeros((3, d, H, W), np.float64)
        self._lib.oracle_get_state(self._h, _ptr(P), _ptr(beta))
        return P, beta

    def get_beta(self):
        """beta (3,d,H,W) alone."""
        beta = np.zeros((3, self.d, self.H, self.W), np.float64)
        self._lib.oracle_get_beta(self._h, _ptr(beta))
        return beta

    def get_history(self):
        """Paper mode: the temporal feature history z, (3,H,W)."""
        z = np.zeros((3, self.H, self.W), np.float64)
        self._lib.oracle_get_history(self._h, _ptr(z))
        return z

    def set_history(self, z):
        z = _f64(z, (3, self.H, self.W))
        self._lib.oracle_set_history(self._h, _ptr(z))

    def set_state(self, P, beta, frames=1):
        W, H, d = self.W, self.H, self.d
        P = _f64(P, (d, d, H, W))
        beta = _f64(beta, (3, d, H, W))
        self._lib.oracle_set_state(self._h, _ptr(P), _ptr(beta), int(frames))
