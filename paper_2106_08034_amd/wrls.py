"""Python binding of libwrls (include/wrls.h): argument marshalling only.

Every function named like the C ABI (wrls_create_stream, wrls_step, ...)
forwards to the entry point of the same name; torch tensors supply device
memory and torch's current HIP stream supplies the stream.  All arithmetic
runs in the HIP kernels of libwrls.so.  There is no fallback: if the library
is not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwrls.so")

WRLS_OK, WRLS_EINVAL, WRLS_ENOMEM, WRLS_EHIP, WRLS_EUNSUPPORTED = 0, -1, -2, -3, -4
WRLS_F32, WRLS_F16 = 0, 1
WRLS_W_INVVAR, WRLS_W_ONE, WRLS_W_PAPER = 0, 1, 2
WRLS_INTERP_BILINEAR, WRLS_INTERP_NEAREST = 0, 1
WRLS_MAX_D = 10

_STATUS_NAMES = {0: "WRLS_OK", -1: "WRLS_EINVAL", -2: "WRLS_ENOMEM", -3: "WRLS_EHIP",
                 -4: "WRLS_EUNSUPPORTED"}


class WrlsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class wrls_params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("d", ctypes.c_int32),
                ("lambda_", ctypes.c_float), ("delta", ctypes.c_float),
                ("var_floor", ctypes.c_float), ("in_dtype", ctypes.c_int32),
                ("weight_mode", ctypes.c_int32), ("interp", ctypes.c_int32),
                ("alpha", ctypes.c_float), ("h", ctypes.c_float), ("eps", ctypes.c_float),
                ("sigma0", ctypes.c_float), ("lambda_min", ctypes.c_float)]


class wrls_frame(ctypes.Structure):
    _fields_ = [("color", ctypes.c_void_p), ("features", ctypes.c_void_p),
                ("variance", ctypes.c_void_p), ("motion", ctypes.c_void_p), ("out", ctypes.c_void_p)]


WRLS_MAX_BATCH = 64
WRLS_NOALLOC_MAX_STREAMS = 64

# Every symbol include/wrls.h declares, with its ctypes signature.
_P = ctypes.POINTER(wrls_params)
_VP = ctypes.c_void_p
SIGNATURES = {
    "wrls_params_default": (None, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "wrls_params_validate": (ctypes.c_int, [_P]),
    "wrls_state_floats": (ctypes.c_int32, [ctypes.c_int32]),
    "wrls_state_bytes": (ctypes.c_size_t, [_P]),
    "wrls_stream_device_bytes": (ctypes.c_size_t, [_P]),
    "wrls_create_stream": (ctypes.c_int, [_P, _VP, ctypes.POINTER(_VP)]),
    "wrls_create_stream_in": (ctypes.c_int, [_P, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "wrls_destroy": (ctypes.c_int, [_VP]),
    "wrls_set_hip_stream": (ctypes.c_int, [_VP, _VP]),
    "wrls_set_tile": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "wrls_get_tile": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "wrls_reset": (ctypes.c_int, [_VP]),
    "wrls_frames": (ctypes.c_int64, [_VP]),
    "wrls_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "wrls_get_state": (ctypes.c_int, [_VP, _VP, _VP]),
    "wrls_set_state": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64]),
    "wrls_blend": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_float, ctypes.c_float, _VP]),
    "wrls_get_history": (ctypes.c_int, [_VP, _VP]),
    "wrls_set_history": (ctypes.c_int, [_VP, _VP]),
    "wrls_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                         ctypes.POINTER(_VP)]),
    "wrls_batch_destroy": (ctypes.c_int, [_VP]),
    "wrls_batch_hip_stream": (_VP, [_VP]),
    "wrls_batch_set_tile": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "wrls_batch_use_graph": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "wrls_batch_step": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(_VP),
                                       ctypes.POINTER(wrls_frame)]),
    "wrls_batch_step_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_VP),
                                               ctypes.POINTER(wrls_frame), ctypes.c_int32,
                                               ctypes.c_int32, _VP]),
    "wrls_traffic_probe": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "wrls_checked_build": (ctypes.c_int32, []),
    "wrls_checked_failures": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint32)]),
    "wrls_checked_raise": (ctypes.c_int, [ctypes.c_uint32, _VP]),
    "wrls_device_copy": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP]),
    "wrls_last_error": (ctypes.c_char_p, []),
    "wrls_version": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libwrls.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwrls.so is not built: run __graft_entry__.build() or "
                          "python paper_2106_08034_amd/build.py")
    # torch loads its own HIP runtime (soname libamdhip64.so.7) under another
    # file name; loading torch first makes libwrls bind to that same runtime
    # instead of pulling a second copy into the process.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != WRLS_OK:
        raise WrlsError(status, lib().wrls_last_error().decode(errors="replace"))


# ---- the C ABI, name for name -------------------------------------------

def wrls_params_default(width: int, height: int, d: int) -> wrls_params:
    p = wrls_params()
    lib().wrls_params_default(ctypes.byref(p), width, height, d)
    return p


def wrls_params_validate(p: wrls_params) -> int:
    return lib().wrls_params_validate(ctypes.byref(p))


def wrls_state_floats(d: int) -> int:
    return lib().wrls_state_floats(d)


def wrls_state_bytes(p: wrls_params) -> int:
    return lib().wrls_state_bytes(ctypes.byref(p))


def wrls_stream_device_bytes(p: wrls_params) -> int:
    return lib().wrls_stream_device_bytes(ctypes.byref(p))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _current_hip_stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


def wrls_create_stream(p: wrls_params, hip_stream: Optional[int] = None) -> int:
    h = ctypes.c_void_p()
    _check(lib().wrls_create_stream(ctypes.byref(p), hip_stream, ctypes.byref(h)))
    return h.value


def wrls_create_stream_in(p: wrls_params, device_mem: int, nbytes: int,
                          hip_stream: Optional[int] = None) -> int:
    h = ctypes.c_void_p()
    _check(lib().wrls_create_stream_in(ctypes.byref(p), device_mem, nbytes, hip_stream,
                                       ctypes.byref(h)))
    return h.value


def wrls_destroy(h: int):
    _check(lib().wrls_destroy(h))


def wrls_set_hip_stream(h: int, hip_stream: Optional[int]):
    _check(lib().wrls_set_hip_stream(h, hip_stream))


def wrls_set_tile(h: int, tile_w_log2: int, block_threads: int, strip_tiles: int = 0):
    _check(lib().wrls_set_tile(h, tile_w_log2, block_threads, strip_tiles))


def wrls_get_tile(h: int) -> Tuple[int, int, int]:
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().wrls_get_tile(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def wrls_reset(h: int):
    _check(lib().wrls_reset(h))


def wrls_frames(h: int) -> int:
    return lib().wrls_frames(h)


def wrls_step(h: int, color, features, variance, motion, out):
    _check(lib().wrls_step(h, _ptr(color), _ptr(features), _ptr(variance), _ptr(motion),
                           _ptr(out)))


def wrls_traffic_probe(h: int, color, features, variance, motion, out):
    _check(lib().wrls_traffic_probe(h, _ptr(color), _ptr(features), _ptr(variance), _ptr(motion),
                                    _ptr(out)))


CHECK_SITES = ("gather tap", "state or output store", "blend halo load", "blend LDS index",
               "paper-mode LDS index", "batched tile without a frame")


def wrls_checked_build() -> int:
    """1 if the loaded library is the checked build, 0 if the shipped one."""
    return int(lib().wrls_checked_build())


def wrls_checked_raise(site_mask: int, hip_stream: Optional[int] = None):
    """Checked builds: fails the checks of the sites in site_mask from a
    kernel (to exercise the reporting path)."""
    st = _current_hip_stream() if hip_stream is None else hip_stream
    _check(lib().wrls_checked_raise(site_mask, st))


def wrls_checked_failures() -> int:
    """Checked builds: the bit mask of the sites whose access checks failed
    since the last call (and clears them); 0 = every access in bounds."""
    m = ctypes.c_uint32(0)
    _check(lib().wrls_checked_failures(ctypes.byref(m)))
    return m.value


def wrls_get_state(h: int, P_packed, beta):
    _check(lib().wrls_get_state(h, _ptr(P_packed), _ptr(beta)))


def wrls_set_state(h: int, P_packed, beta, frames: int):
    _check(lib().wrls_set_state(h, _ptr(P_packed), _ptr(beta), frames))


def wrls_batch_create(max_streams: int, d: int, in_dtype: int,
                      hip_stream: Optional[int] = None) -> int:
    h = ctypes.c_void_p()
    _check(lib().wrls_batch_create(max_streams, d, in_dtype, hip_stream, ctypes.byref(h)))
    return h.value


def wrls_batch_destroy(b: int):
    _check(lib().wrls_batch_destroy(b))


def wrls_batch_hip_stream(b: int) -> Optional[int]:
    return lib().wrls_batch_hip_stream(b)


def wrls_batch_set_tile(b: int, tile_w_log2: int, block_threads: int, blocks_per_cu: int):
    _check(lib().wrls_batch_set_tile(b, tile_w_log2, block_threads, blocks_per_cu))


def wrls_batch_use_graph(b: int, enable: bool):
    _check(lib().wrls_batch_use_graph(b, int(bool(enable))))


def wrls_batch_step(b: int, handles, frames):
    """handles: stream handles; frames: tuples (color, features, variance,
    motion, out) of tensors (or None)."""
    n = len(handles)
    hs = (ctypes.c_void_p * max(n, 1))(*handles)
    fs = (wrls_frame * max(n, 1))(*[wrls_frame(*[_ptr(t) for t in f]) for f in frames])
    _check(lib().wrls_batch_step(b, n, hs, fs))


def wrls_batch_step_noalloc(handles, frames, tile_w_log2: int = 7, block_threads: int = 128,
                            hip_stream: Optional[int] = None):
    """One batched step that allocates nothing (the frame table is the
    library's fixed per-device array); handles and frames as in
    wrls_batch_step; hip_stream None: torch's current stream."""
    n = len(handles)
    hs = (ctypes.c_void_p * max(n, 1))(*handles)
    fs = (wrls_frame * max(n, 1))(*[wrls_frame(*[_ptr(t) for t in f]) for f in frames])
    st = _current_hip_stream() if hip_stream is None else hip_stream
    _check(lib().wrls_batch_step_noalloc(n, hs, fs, tile_w_log2, block_threads, st))


def wrls_blend(h: int, features, temporal, sigma_s: float, sigma_r: float, out):
    _check(lib().wrls_blend(h, _ptr(features), _ptr(temporal), float(sigma_s), float(sigma_r),
                            _ptr(out)))


def wrls_get_history(h: int, z):
    _check(lib().wrls_get_history(h, _ptr(z)))


def wrls_set_history(h: int, z):
    _check(lib().wrls_set_history(h, _ptr(z)))


def wrls_device_copy(dst, src, nbytes: Optional[int] = None, hip_stream: Optional[int] = None):
    """Copies nbytes (default: all of src) from tensor src to tensor dst on
    the library's 16-byte copy kernel, on torch's current stream unless
    hip_stream is given."""
    n = src.numel() * src.element_size() if nbytes is None else nbytes
    hs = _current_hip_stream() if hip_stream is None else hip_stream
    _check(lib().wrls_device_copy(_ptr(dst), _ptr(src), n, hs))


def wrls_last_error() -> str:
    return lib().wrls_last_error().decode(errors="replace")


def wrls_version() -> str:
    return lib().wrls_version().decode()


# ---- convenience wrapper over torch tensors -------------------------------

_DTYPES = {"f32": WRLS_F32, "f16": WRLS_F16}
_WMODES = {"invvar": WRLS_W_INVVAR, "one": WRLS_W_ONE, "paper": WRLS_W_PAPER}
_INTERPS = {"bilinear": WRLS_INTERP_BILINEAR, "nearest": WRLS_INTERP_NEAREST}


def make_params(width, height, d, lam=0.98, delta=1.0, var_floor=1e-6, in_dtype="f32",
                weight_mode="invvar", interp="bilinear", alpha=0.75, h=0.75,
                eps=1e-4, sigma0=0.0, lam_min=0.0) -> wrls_params:
    p = wrls_params_default(width, height, d)
    p.lambda_, p.delta, p.var_floor = lam, delta, var_floor
    p.in_dtype, p.weight_mode, p.interp = _DTYPES[in_dtype], _WMODES[weight_mode], _INTERPS[interp]
    p.alpha, p.h, p.eps = alpha, h, eps
    p.sigma0, p.lambda_min = sigma0, lam_min
    return p


class Stream:
    """One image sequence whose per-pixel models live on the GPU.

    All work is enqueued on the torch stream current at creation (or the
    one passed); tensors must be contiguous, on the current device, with the
    shapes documented in include/wrls.h.
    """

    def __init__(self, width: int, height: int, d: int, lam: float = 0.98, delta: float = 1.0,
                 var_floor: float = 1e-6, in_dtype: str = "f32", weight_mode: str = "invvar",
                 interp: str = "bilinear", hip_stream: Optional[int] = None,
                 device_mem: Optional[Tuple[int, int]] = None, alpha: float = 0.75,
                 h: float = 0.75, eps: float = 1e-4, sigma0: float = 0.0, lam_min: float = 0.0):
        """device_mem: (pointer, bytes) of caller-owned device memory for the
        state (wrls_create_stream_in); None: the library allocates.
        weight_mode "paper" (d = 4): the paper's predictor and weight
        (alpha, h, eps); features and variance are then not used.
        sigma0 > 0: automatic forgetting factor in [lam_min, lam]."""
        import torch
        self._torch = torch
        p = make_params(width, height, d, lam, delta, var_floor, in_dtype, weight_mode, interp,
                        alpha, h, eps, sigma0, lam_min)
        self.paper = weight_mode == "paper"
        self.params = p
        self.W, self.H, self.d = width, height, d
        self.in_dtype = torch.float16 if in_dtype == "f16" else torch.float32
        self.hip_stream = _current_hip_stream() if hip_stream is None else hip_stream
        if device_mem is None:
            self.handle = wrls_create_stream(p, self.hip_stream)
        else:
            self.handle = wrls_create_stream_in(p, device_mem[0], device_mem[1], self.hip_stream)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the runtime may be gone
            pass

    def close(self):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            wrls_destroy(h)

    @property
    def frames(self) -> int:
        return wrls_frames(self.handle)

    def _chk(self, t, shape, dtype, name):
        if t is None:
            return None
        if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError("%s: expected contiguous %s %s on the GPU, got %s %s %s"
                             % (name, dtype, tuple(shape), t.dtype, tuple(t.shape), t.device))
        return t

    def step(self, color, features, variance, motion=None, out=None):
        torch = self._torch
        W, H, d = self.W, self.H, self.d
        self._chk(color, (3, H, W), self.in_dtype, "color")
        if d > 1 and not self.paper:
            self._chk(features, (d - 1, H, W), self.in_dtype, "features")
        self._chk(variance, (H, W), torch.float32, "variance")
        self._chk(motion, (2, H, W), torch.float32, "motion")
        if out is None:
            out = torch.empty((3, H, W), dtype=torch.float32, device=color.device)
        self._chk(out, (3, H, W), torch.float32, "out")
        wrls_step(self.handle, color, features if (d > 1 and not self.paper) else None, variance,
                  motion, out)
        return out

    def traffic_probe(self, color, features, variance, motion=None, out=None):
        """wrls_traffic_probe: the step's loads and stores without the
        reprojection and the arithmetic (a measurement reference; the
        stream's state is left as it was, and out holds no result)."""
        torch = self._torch
        W, H, d = self.W, self.H, self.d
        self._chk(color, (3, H, W), self.in_dtype, "color")
        if d > 1 and not self.paper:
            self._chk(features, (d - 1, H, W), self.in_dtype, "features")
        self._chk(variance, (H, W), torch.float32, "variance")
        self._chk(motion, (2, H, W), torch.float32, "motion")
        if out is None:
            out = torch.empty((3, H, W), dtype=torch.float32, device=color.device)
        self._chk(out, (3, H, W), torch.float32, "out")
        wrls_traffic_probe(self.handle, color, features if (d > 1 and not self.paper) else None,
                           variance, motion, out)
        return out

    def reset(self):
        wrls_reset(self.handle)

    def set_tile(self, tile_w_log2: int, block_threads: int, strip_tiles: int = 0):
        wrls_set_tile(self.handle, tile_w_log2, block_threads, strip_tiles)

    @property
    def tile(self) -> Tuple[int, int, int]:
        return wrls_get_tile(self.handle)

    def get_state(self) -> Tuple["object", "object"]:
        torch = self._torch
        W, H, d = self.W, self.H, self.d
        P = torch.empty((d * (d + 1) // 2, H, W), dtype=torch.float32, device="cuda")
        B = torch.empty((3, d, H, W), dtype=torch.float32, device="cuda")
        wrls_get_state(self.handle, P, B)
        return P, B

    def blend(self, features, temporal, sigma_s: float, sigma_r: float, out=None):
        """The 5x5 spatial blend (wrls_blend) on the current state: features
        of the last step (ignored in paper mode), temporal = that step's
        output.  Returns the blended (3, H, W) image."""
        torch = self._torch
        W, H, d = self.W, self.H, self.d
        use_f = d > 1 and not self.paper
        if use_f:
            self._chk(features, (d - 1, H, W), self.in_dtype, "features")
        self._chk(temporal, (3, H, W), torch.float32, "temporal")
        if out is None:
            out = torch.empty((3, H, W), dtype=torch.float32, device=temporal.device)
        self._chk(out, (3, H, W), torch.float32, "out")
        wrls_blend(self.handle, features if use_f else None, temporal, sigma_s, sigma_r, out)
        return out

    def get_history(self):
        """Paper mode: the temporal feature history z, (3, H, W)."""
        z = self._torch.empty((3, self.H, self.W), dtype=self._torch.float32, device="cuda")
        wrls_get_history(self.handle, z)
        return z

    def set_history(self, z):
        self._chk(z, (3, self.H, self.W), self._torch.float32, "z")
        wrls_set_history(self.handle, z)

    def set_state(self, P_packed, beta, frames: int = 1):
        torch = self._torch
        W, H, d = self.W, self.H, self.d
        self._chk(P_packed, (d * (d + 1) // 2, H, W), torch.float32, "P_packed")
        self._chk(beta, (3, d, H, W), torch.float32, "beta")
        wrls_set_state(self.handle, P_packed, beta, frames)


class Batch:
    """Advances several Streams by one frame each with one persistent
    launch (optionally a replayed HIP graph) on the batch's HIP stream."""

    def __init__(self, max_streams: int, d: int, in_dtype: str = "f32",
                 hip_stream: Optional[int] = None, use_graph: bool = True):
        import torch
        self._torch = torch
        self.d = d
        self.in_dtype = in_dtype
        hs = _current_hip_stream() if hip_stream is None else hip_stream
        self.handle = wrls_batch_create(max_streams, d, _DTYPES[in_dtype], hs)
        self.hip_stream = wrls_batch_hip_stream(self.handle)
        wrls_batch_use_graph(self.handle, use_graph)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            wrls_batch_destroy(h)

    def set_tile(self, tile_w_log2: int, block_threads: int, blocks_per_cu: int):
        wrls_batch_set_tile(self.handle, tile_w_log2, block_threads, blocks_per_cu)

    def use_graph(self, enable: bool):
        wrls_batch_use_graph(self.handle, enable)

    def step(self, streams, frames, outs=None):
        """streams: list of Stream; frames: list of (color, features,
        variance, motion) tensors; outs: optional output tensors.  Returns
        the output tensors."""
        torch = self._torch
        if outs is None:
            outs = [torch.empty((3, s.H, s.W), dtype=torch.float32, device="cuda") for s in streams]
        full = []
        for s, f, o in zip(streams, frames, outs):
            c, fe, v, m = f
            s._chk(c, (3, s.H, s.W), s.in_dtype, "color")
            if s.d > 1:
                s._chk(fe, (s.d - 1, s.H, s.W), s.in_dtype, "features")
            s._chk(v, (s.H, s.W), torch.float32, "variance")
            s._chk(m, (2, s.H, s.W), torch.float32, "motion")
            s._chk(o, (3, s.H, s.W), torch.float32, "out")
            full.append((c, fe if s.d > 1 else None, v, m, o))
        wrls_batch_step(self.handle, [s.handle for s in streams], full)
        return outs
