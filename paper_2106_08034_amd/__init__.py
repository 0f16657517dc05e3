"""MI355X-native per-pixel weighted recursive least squares (wRLS) temporal
denoiser (Iglesias-Guitian, Mane and Moon, IEEE TVCG 2020, Sec. 5).

The arithmetic lives in hand-written HIP kernels for gfx950 behind the C ABI
of include/wrls.h (libwrls.so); `wrls` is its Python binding.
"""
from . import wrls  # noqa: F401
from .wrls import Stream, WrlsError  # noqa: F401
