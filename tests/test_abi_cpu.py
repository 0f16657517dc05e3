"""The C ABI without a GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments with status codes before any HIP
call is made."""
import ctypes
import os
import re
import threading

import pytest

from paper_2106_08034_amd import wrls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wrls.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(wrls_\w+)\s*\(", src, flags=re.M))


def test_header_symbols_exported_and_bound():
    names = _declared()
    assert {"wrls_create_stream", "wrls_step", "wrls_destroy"} <= names
    L = wrls.lib()
    for n in sorted(names):
        assert hasattr(L, n), "libwrls.so does not export %s" % n
        assert n in wrls.SIGNATURES, "the binding does not declare %s" % n
        assert callable(getattr(wrls, n)), "the binding has no function %s" % n
    assert set(wrls.SIGNATURES) == names


def test_state_sizes():
    for d in range(1, 11):
        assert wrls.wrls_state_floats(d) == d * (d + 1) // 2 + 3 * d
    assert wrls.wrls_state_floats(0) == 0
    assert wrls.wrls_state_floats(11) == 0
    p = wrls.wrls_params_default(1920, 1080, 8)
    assert wrls.wrls_state_bytes(p) == 240 * 1920 * 1080
    assert wrls.wrls_stream_device_bytes(p) >= 2 * 240 * 1920 * 1080
    p = wrls.wrls_params_default(3840, 2160, 10)
    assert wrls.wrls_state_bytes(p) == 340 * 3840 * 2160


def test_defaults():
    p = wrls.wrls_params_default(64, 48, 8)
    assert (p.width, p.height, p.d) == (64, 48, 8)
    assert abs(p.lambda_ - 0.98) < 1e-7 and p.delta == 1.0 and abs(p.var_floor - 1e-6) < 1e-12
    assert p.in_dtype == wrls.WRLS_F32 and p.weight_mode == wrls.WRLS_W_INVVAR
    assert p.interp == wrls.WRLS_INTERP_BILINEAR
    assert wrls.wrls_params_validate(p) == wrls.WRLS_OK


@pytest.mark.parametrize("field,value,status", [
    ("width", 0, wrls.WRLS_EINVAL), ("height", 16385, wrls.WRLS_EINVAL),
    ("width", -3, wrls.WRLS_EINVAL), ("d", 0, wrls.WRLS_EUNSUPPORTED),
    ("d", 11, wrls.WRLS_EUNSUPPORTED), ("lambda_", 0.0, wrls.WRLS_EINVAL),
    ("lambda_", 1.5, wrls.WRLS_EINVAL), ("lambda_", float("nan"), wrls.WRLS_EINVAL),
    ("delta", 0.0, wrls.WRLS_EINVAL), ("delta", float("inf"), wrls.WRLS_EINVAL),
    ("var_floor", -1.0, wrls.WRLS_EINVAL), ("in_dtype", 7, wrls.WRLS_EINVAL),
    ("weight_mode", 5, wrls.WRLS_EINVAL), ("interp", 2, wrls.WRLS_EINVAL),
])
def test_bad_params_rejected_without_gpu(field, value, status):
    p = wrls.wrls_params_default(64, 48, 8)
    setattr(p, field, value)
    assert wrls.wrls_params_validate(p) == status
    assert wrls.wrls_last_error()
    assert wrls.wrls_state_bytes(p) == 0
    h = ctypes.c_void_p(123)
    rc = wrls.lib().wrls_create_stream(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == status and h.value is None


def test_state_copy_limit_4gib():
    p = wrls.wrls_params_default(16384, 16384, 10)
    assert wrls.wrls_params_validate(p) == wrls.WRLS_EUNSUPPORTED
    assert "4 GiB" in wrls.wrls_last_error()
    p = wrls.wrls_params_default(3840, 2160, 10)
    assert wrls.wrls_params_validate(p) == wrls.WRLS_OK
    # the largest square image at d = 10 whose state copy fits; planes are
    # an odd number of 256-byte units apart
    S = wrls.wrls_state_floats(10)

    def pitch(npix):
        q = (npix + 63) // 64
        return (q + 1 - q % 2) * 64

    side = int(((2 ** 32 - 1) // (4 * S)) ** 0.5) // 8 * 8
    while pitch(side * side) * 4 * S > 2 ** 32 - 1:
        side -= 8
    assert wrls.wrls_params_validate(wrls.wrls_params_default(side, side, 10)) == wrls.WRLS_OK
    assert wrls.wrls_params_validate(wrls.wrls_params_default(side + 64, side + 64, 10)) == wrls.WRLS_EUNSUPPORTED
    p = wrls.wrls_params_default(2560, 1440, 8)
    assert wrls.wrls_stream_device_bytes(p) == 2 * 60 * 4 * pitch(2560 * 1440) + 256


def test_paper_mode_parameters():
    p = wrls.wrls_params_default(64, 48, 4)
    assert abs(p.alpha - 0.75) < 1e-7 and abs(p.h - 0.75) < 1e-7 and abs(p.eps - 1e-4) < 1e-9
    p.weight_mode = wrls.WRLS_W_PAPER
    assert wrls.wrls_params_validate(p) == wrls.WRLS_OK
    # the history adds 3 entries per pixel
    assert wrls.wrls_state_bytes(p) == (10 + 12 + 3) * 4 * 64 * 48
    p.d = 8
    assert wrls.wrls_params_validate(p) == wrls.WRLS_EINVAL and "d = 4" in wrls.wrls_last_error()
    p.d = 4
    for field, bad in (("alpha", 1.5), ("alpha", -0.1), ("h", 0.0), ("h", float("inf")), ("h", 1e-25),
                       ("eps", -1.0), ("eps", 0.0), ("eps", float("nan"))):
        q = wrls.wrls_params_default(64, 48, 4)
        q.weight_mode = wrls.WRLS_W_PAPER
        setattr(q, field, bad)
        assert wrls.wrls_params_validate(q) == wrls.WRLS_EINVAL, (field, bad)
    L = wrls.lib()
    assert L.wrls_get_history(None, None) == wrls.WRLS_EINVAL
    assert L.wrls_set_history(None, None) == wrls.WRLS_EINVAL


def test_automatic_forgetting_parameters():
    """sigma0 = 0 (the default) fixes lambda; sigma0 > 0 or +inf turns the
    automatic factor on and needs lambda_min in (0, lambda]."""
    p = wrls.wrls_params_default(8, 8, 8)
    assert p.sigma0 == 0.0 and p.lambda_min == 0.0
    assert wrls.wrls_params_validate(p) == wrls.WRLS_OK
    for s0, lo, ok in ((30.0, 0.5, True), (float("inf"), 0.98, True), (30.0, 0.0, False),
                       (30.0, 0.99, False), (-1.0, 0.5, False), (float("nan"), 0.5, False),
                       (30.0, float("nan"), False)):
        q = wrls.wrls_params_default(8, 8, 8)
        q.sigma0, q.lambda_min = s0, lo
        rc = wrls.wrls_params_validate(q)
        assert (rc == wrls.WRLS_OK) == ok, (s0, lo, wrls.wrls_last_error())


def test_null_arguments():
    L = wrls.lib()
    assert L.wrls_params_validate(None) == wrls.WRLS_EINVAL
    p = wrls.wrls_params_default(8, 8, 8)
    assert L.wrls_create_stream(ctypes.byref(p), None, None) == wrls.WRLS_EINVAL
    assert L.wrls_destroy(None) == wrls.WRLS_OK
    assert L.wrls_reset(None) == wrls.WRLS_EINVAL
    assert L.wrls_frames(None) == -1
    assert L.wrls_step(None, None, None, None, None, None) == wrls.WRLS_EINVAL
    assert L.wrls_get_state(None, None, None) == wrls.WRLS_EINVAL
    assert L.wrls_set_state(None, None, None, 0) == wrls.WRLS_EINVAL
    assert L.wrls_set_hip_stream(None, None) == wrls.WRLS_EINVAL
    assert L.wrls_set_tile(None, 6, 256, 0) == wrls.WRLS_EINVAL
    assert L.wrls_get_tile(None, None, None, None) == wrls.WRLS_EINVAL
    assert L.wrls_blend(None, None, None, 1.0, 1.0, None) == wrls.WRLS_EINVAL
    assert L.wrls_traffic_probe(None, None, None, None, None, None) == wrls.WRLS_EINVAL
    L.wrls_params_default(None, 1, 1, 1)  # ignored, must not crash
    with pytest.raises(wrls.WrlsError):
        wrls.wrls_reset(None)


def test_last_error_is_thread_local():
    p = wrls.wrls_params_default(8, 8, 8)
    p.d = 99
    wrls.wrls_params_validate(p)
    mine = wrls.wrls_last_error()
    seen = []
    t = threading.Thread(target=lambda: seen.append(wrls.wrls_last_error()))
    t.start()
    t.join()
    assert "d = 99" in mine and seen == [""]


def test_batch_and_stream_in_reject_bad_arguments_without_gpu():
    L = wrls.lib()
    h = ctypes.c_void_p()
    assert L.wrls_batch_create(0, 8, 0, None, ctypes.byref(h)) == wrls.WRLS_EINVAL
    assert L.wrls_batch_create(wrls.WRLS_MAX_BATCH + 1, 8, 0, None, ctypes.byref(h)) == wrls.WRLS_EINVAL
    assert L.wrls_batch_create(4, 11, 0, None, ctypes.byref(h)) == wrls.WRLS_EUNSUPPORTED
    assert L.wrls_batch_create(4, 8, 3, None, ctypes.byref(h)) == wrls.WRLS_EINVAL
    assert L.wrls_batch_create(4, 8, 0, None, None) == wrls.WRLS_EINVAL
    assert L.wrls_batch_destroy(None) == wrls.WRLS_OK
    assert L.wrls_batch_step(None, 0, None, None) == wrls.WRLS_EINVAL
    assert L.wrls_batch_set_tile(None, 7, 256, 5) == wrls.WRLS_EINVAL
    assert L.wrls_batch_use_graph(None, 1) == wrls.WRLS_EINVAL
    assert L.wrls_batch_hip_stream(None) is None
    p = wrls.wrls_params_default(64, 48, 8)
    need = wrls.wrls_stream_device_bytes(p)
    assert L.wrls_create_stream_in(ctypes.byref(p), None, need, None, ctypes.byref(h)) == wrls.WRLS_EINVAL
    # checked before any device access: misaligned or too small regions
    assert L.wrls_create_stream_in(ctypes.byref(p), ctypes.c_void_p(0x1000 + 4), need, None,
                                   ctypes.byref(h)) == wrls.WRLS_EINVAL
    assert "aligned" in wrls.wrls_last_error()
    assert L.wrls_create_stream_in(ctypes.byref(p), ctypes.c_void_p(0x1000), need - 1, None,
                                   ctypes.byref(h)) == wrls.WRLS_EINVAL
    assert "needs" in wrls.wrls_last_error()


def test_checked_library_exports_the_same_abi():
    """libwrls_checked.so (the kernels' access checks compiled in) exports
    every symbol of the header and says it is the checked build; the
    shipped library says it is not and has no check flags to read."""
    import os
    C = ctypes.CDLL(os.path.join(os.path.dirname(wrls.LIB_PATH), "libwrls_checked.so"))
    for n in sorted(_declared()):
        assert hasattr(C, n), "libwrls_checked.so does not export %s" % n
    C.wrls_checked_build.restype = ctypes.c_int32
    assert C.wrls_checked_build() == 1
    assert wrls.wrls_checked_build() == 0
    m = ctypes.c_uint32(7)
    assert wrls.lib().wrls_checked_failures(ctypes.byref(m)) == wrls.WRLS_EUNSUPPORTED
    assert m.value == 7
    assert "without checks" in wrls.wrls_last_error()
    assert wrls.lib().wrls_checked_raise(1, None) == wrls.WRLS_EUNSUPPORTED


def test_device_copy_rejects_bad_arguments_on_the_host():
    """wrls_device_copy validates before any HIP call: null pointers,
    misalignment, a size that is not a multiple of 16 and overlap are
    rejected; zero bytes is a no-op.  (Fake addresses: nothing is launched.)"""
    L = wrls.lib()
    assert L.wrls_device_copy(None, None, 0, None) == wrls.WRLS_OK
    assert L.wrls_device_copy(None, 4096, 16, None) == wrls.WRLS_EINVAL
    assert L.wrls_device_copy(4096, None, 16, None) == wrls.WRLS_EINVAL
    assert L.wrls_device_copy(4096 + 4, 8192, 16, None) == wrls.WRLS_EINVAL   # dst misaligned
    assert L.wrls_device_copy(4096, 8192 + 8, 16, None) == wrls.WRLS_EINVAL   # src misaligned
    assert L.wrls_device_copy(4096, 8192, 24, None) == wrls.WRLS_EINVAL       # not whole vectors
    assert L.wrls_device_copy(4096, 4096 + 32, 64, None) == wrls.WRLS_EINVAL  # overlap
    assert L.wrls_device_copy(4096 + 32, 4096, 64, None) == wrls.WRLS_EINVAL
    assert "overlap" in wrls.wrls_last_error()


def test_noalloc_step_rejects_beyond_its_table_on_the_host():
    """The allocation-free batched step holds at most WRLS_NOALLOC_MAX_STREAMS
    frames in its fixed table: more (or a negative count, or a bad tile) is
    refused before anything reaches the GPU; n = 0 is a no-op."""
    L = wrls.lib()
    assert wrls.WRLS_NOALLOC_MAX_STREAMS == 64
    assert L.wrls_batch_step_noalloc(65, None, None, 7, 128, None) == wrls.WRLS_EINVAL
    assert "65" in wrls.wrls_last_error() and "64" in wrls.wrls_last_error()
    assert L.wrls_batch_step_noalloc(-1, None, None, 7, 128, None) == wrls.WRLS_EINVAL
    assert L.wrls_batch_step_noalloc(0, None, None, 7, 128, None) == wrls.WRLS_OK
    assert L.wrls_batch_step_noalloc(1, None, None, 7, 128, None) == wrls.WRLS_EINVAL
    hs = (ctypes.c_void_p * 1)(None)
    fs = (wrls.wrls_frame * 1)()
    assert L.wrls_batch_step_noalloc(1, hs, fs, 8, 128, None) == wrls.WRLS_EINVAL   # tile too wide
    assert L.wrls_batch_step_noalloc(1, hs, fs, 7, 96, None) == wrls.WRLS_EINVAL
    assert L.wrls_batch_step_noalloc(1, hs, fs, 7, 128, None) == wrls.WRLS_EINVAL   # NULL stream
