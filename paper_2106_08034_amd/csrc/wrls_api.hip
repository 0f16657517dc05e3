// C ABI of libwrls (declared in include/wrls.h): argument checking, state
// ownership and launches.  No exception leaves this file; every failure is a
// status code plus a thread-local message.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "wrls.h"
#include "wrls_internal.h"

struct wrls_stream {
    wrls_params prm;
    hipStream_t st;
    float *state[2];  // previous / current frame, S planes of `pitch` floats each
    void *alloc;      // the single device allocation holding both copies
    int64_t pitch;
    int cur;          // index of the state holding the latest frame
    int64_t frames;
    wrls::TileShape tile;
};

namespace {

thread_local char g_err[512];

wrls_status fail(wrls_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

wrls_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? WRLS_ENOMEM : WRLS_EHIP, "%s: %s (%d)", what,
                hipGetErrorString(e), (int)e);
}

int64_t plane_pitch(const wrls_params *p)
{
    const int64_t n = (int64_t)p->width * p->height;
    const int64_t a = (int64_t)wrls::kPlaneAlign;
    return (n + a - 1) / a * a;
}

wrls::TileShape default_tile() { return wrls::TileShape{7, 256, 0}; }

}  // namespace

extern "C" {

void wrls_params_default(wrls_params *p, int32_t width, int32_t height, int32_t d)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->width = width;
    p->height = height;
    p->d = d;
    p->lambda = 0.98f;
    p->delta = 1.0f;
    p->var_floor = 1e-6f;
    p->in_dtype = WRLS_F32;
    p->weight_mode = WRLS_W_INVVAR;
    p->interp = WRLS_INTERP_BILINEAR;
}

wrls_status wrls_params_validate(const wrls_params *p)
{
    if (!p) return fail(WRLS_EINVAL, "params is NULL");
    if (p->width < 1 || p->height < 1 || p->width > 16384 || p->height > 16384)
        return fail(WRLS_EINVAL, "image size %dx%d outside [1, 16384]", p->width, p->height);
    if (p->d < 1 || p->d > WRLS_MAX_D)
        return fail(WRLS_EUNSUPPORTED, "d = %d outside [1, %d]", p->d, WRLS_MAX_D);
    if (!(p->lambda > 0.0f && p->lambda <= 1.0f))
        return fail(WRLS_EINVAL, "lambda = %g outside (0, 1]", (double)p->lambda);
    if (!(p->delta > 0.0f) || !std::isfinite(p->delta))
        return fail(WRLS_EINVAL, "delta = %g must be finite and > 0", (double)p->delta);
    if (!(p->var_floor >= 0.0f) || !std::isfinite(p->var_floor))
        return fail(WRLS_EINVAL, "var_floor = %g must be finite and >= 0", (double)p->var_floor);
    if (p->in_dtype != WRLS_F32 && p->in_dtype != WRLS_F16)
        return fail(WRLS_EINVAL, "in_dtype = %d unknown", p->in_dtype);
    if (p->weight_mode != WRLS_W_INVVAR && p->weight_mode != WRLS_W_ONE)
        return fail(WRLS_EINVAL, "weight_mode = %d unknown", p->weight_mode);
    if (p->interp != WRLS_INTERP_BILINEAR && p->interp != WRLS_INTERP_NEAREST)
        return fail(WRLS_EINVAL, "interp = %d unknown", p->interp);
    for (int i = 0; i < 3; i++)
        if (p->reserved[i] != 0) return fail(WRLS_EINVAL, "reserved fields must be zero");
    // The kernels address every array with 32-bit byte offsets; the state
    // copy is the largest array of a stream.
    const uint64_t copy = (uint64_t)wrls::state_floats(p->d) * sizeof(float) *
                          (uint64_t)plane_pitch(p);
    if (copy > 0xFFFFFFFFull)
        return fail(WRLS_EUNSUPPORTED,
                    "%dx%d at d = %d needs %llu bytes per state copy; the limit is 4 GiB - 1",
                    p->width, p->height, p->d, (unsigned long long)copy);
    return WRLS_OK;
}

int32_t wrls_state_floats(int32_t d)
{
    if (d < 1 || d > WRLS_MAX_D) return 0;
    return wrls::state_floats(d);
}

size_t wrls_state_bytes(const wrls_params *p)
{
    if (wrls_params_validate(p) != WRLS_OK) return 0;
    return (size_t)wrls::state_floats(p->d) * sizeof(float) * (size_t)p->width * (size_t)p->height;
}

size_t wrls_stream_device_bytes(const wrls_params *p)
{
    if (wrls_params_validate(p) != WRLS_OK) return 0;
    return 2 * (size_t)wrls::state_floats(p->d) * sizeof(float) * (size_t)plane_pitch(p);
}

wrls_status wrls_create_stream(const wrls_params *p, void *hip_stream, wrls_stream **out)
{
    if (!out) return fail(WRLS_EINVAL, "out is NULL");
    *out = nullptr;
    wrls_status rc = wrls_params_validate(p);
    if (rc != WRLS_OK) return rc;
    wrls_stream *s = new (std::nothrow) wrls_stream();
    if (!s) return fail(WRLS_ENOMEM, "host allocation of the handle failed");
    s->prm = *p;
    s->st = static_cast<hipStream_t>(hip_stream);
    s->pitch = plane_pitch(p);
    s->cur = 0;
    s->frames = 0;
    s->tile = default_tile();
    const size_t one = (size_t)wrls::state_floats(p->d) * (size_t)s->pitch;
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, 2 * one * sizeof(float));
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipMalloc of the stream state");
    }
    s->alloc = mem;
    s->state[0] = static_cast<float *>(mem);
    s->state[1] = s->state[0] + one;
    const int64_t npix = (int64_t)p->width * p->height;
    e = wrls::launch_reset(s->state[0], s->pitch, npix, p->d, 1.0f / p->delta, s->st);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        delete s;
        return hip_fail(e, "state initialisation");
    }
    *out = s;
    return WRLS_OK;
}

wrls_status wrls_destroy(wrls_stream *s)
{
    if (!s) return WRLS_OK;
    hipError_t e1 = hipStreamSynchronize(s->st);
    hipError_t e2 = hipFree(s->alloc);
    delete s;
    if (e1 != hipSuccess) return hip_fail(e1, "hipStreamSynchronize in destroy");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFree in destroy");
    return WRLS_OK;
}

wrls_status wrls_set_hip_stream(wrls_stream *s, void *hip_stream)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    s->st = static_cast<hipStream_t>(hip_stream);
    return WRLS_OK;
}

wrls_status wrls_set_tile(wrls_stream *s, int32_t tile_w_log2, int32_t block_threads,
                          int32_t strip_tiles)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    if (block_threads != 64 && block_threads != 128 && block_threads != 256)
        return fail(WRLS_EINVAL, "block_threads = %d not in {64, 128, 256}", block_threads);
    if (tile_w_log2 < 0 || (1 << tile_w_log2) > block_threads)
        return fail(WRLS_EINVAL, "tile width 2^%d exceeds %d threads", tile_w_log2, block_threads);
    if (strip_tiles < 0) return fail(WRLS_EINVAL, "strip_tiles = %d < 0", strip_tiles);
    s->tile = wrls::TileShape{tile_w_log2, block_threads, strip_tiles};
    return WRLS_OK;
}

wrls_status wrls_get_tile(const wrls_stream *s, int32_t *tile_w_log2, int32_t *block_threads,
                          int32_t *strip_tiles)
{
    if (!s || !tile_w_log2 || !block_threads || !strip_tiles)
        return fail(WRLS_EINVAL, "NULL argument");
    *tile_w_log2 = s->tile.tw_log2;
    *block_threads = s->tile.block_threads;
    *strip_tiles = s->tile.strip_w;
    return WRLS_OK;
}

wrls_status wrls_reset(wrls_stream *s)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    const int64_t npix = (int64_t)s->prm.width * s->prm.height;
    hipError_t e = wrls::launch_reset(s->state[s->cur], s->pitch, npix, s->prm.d,
                                      1.0f / s->prm.delta, s->st);
    if (e != hipSuccess) return hip_fail(e, "reset launch");
    s->frames = 0;
    return WRLS_OK;
}

int64_t wrls_frames(const wrls_stream *s) { return s ? s->frames : -1; }

wrls_status wrls_step(wrls_stream *s, const void *color, const void *features,
                      const float *variance, const float *motion, float *out)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    const wrls_params &p = s->prm;
    if (!color) return fail(WRLS_EINVAL, "color is NULL");
    if (!out) return fail(WRLS_EINVAL, "out is NULL");
    if (p.d > 1 && !features) return fail(WRLS_EINVAL, "features is NULL with d = %d", p.d);
    if (p.weight_mode == WRLS_W_INVVAR && !variance)
        return fail(WRLS_EINVAL, "variance is NULL with inverse-variance weights");
    wrls::FrameArgs a{};
    a.color = color;
    a.feats = features;
    a.var = p.weight_mode == WRLS_W_INVVAR ? variance : nullptr;
    a.motion = motion;
    a.out = out;
    a.state_in = s->state[s->cur];
    a.state_out = s->state[1 - s->cur];
    a.W = p.width;
    a.H = p.height;
    a.pitch = s->pitch;
    a.lambda = p.lambda;
    a.inv_lambda = 1.0f / p.lambda;
    a.p0 = 1.0f / p.delta;
    a.var_floor = p.var_floor;
    a.fresh = s->frames == 0;
    a.unit_weight = p.weight_mode == WRLS_W_ONE;
    a.nearest = p.interp == WRLS_INTERP_NEAREST;
    hipError_t e = wrls::launch_step(p.d, p.in_dtype == WRLS_F16, a, s->tile, s->st);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    s->cur = 1 - s->cur;
    s->frames++;
    return WRLS_OK;
}

wrls_status wrls_get_state(const wrls_stream *s, float *P_packed, float *beta)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    const int d = s->prm.d;
    const size_t n = (size_t)s->prm.width * s->prm.height;
    const float *src = s->state[s->cur];
    const size_t spitch = (size_t)s->pitch * sizeof(float);
    hipError_t e;
    if (P_packed) {
        e = hipMemcpy2DAsync(P_packed, n * sizeof(float), src, spitch, n * sizeof(float),
                             (size_t)wrls::packed_floats(d), hipMemcpyDeviceToDevice, s->st);
        if (e != hipSuccess) return hip_fail(e, "state export (P)");
    }
    if (beta) {
        e = hipMemcpy2DAsync(beta, n * sizeof(float), src + (size_t)wrls::packed_floats(d) * s->pitch,
                             spitch, n * sizeof(float), (size_t)(3 * d), hipMemcpyDeviceToDevice,
                             s->st);
        if (e != hipSuccess) return hip_fail(e, "state export (beta)");
    }
    return WRLS_OK;
}

wrls_status wrls_set_state(wrls_stream *s, const float *P_packed, const float *beta,
                           int64_t frames)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    if (!P_packed || !beta) return fail(WRLS_EINVAL, "P_packed and beta are both required");
    if (frames < 0) return fail(WRLS_EINVAL, "frames = %lld < 0", (long long)frames);
    const int d = s->prm.d;
    const size_t n = (size_t)s->prm.width * s->prm.height;
    float *dst = s->state[s->cur];
    const size_t dpitch = (size_t)s->pitch * sizeof(float);
    hipError_t e = hipMemcpy2DAsync(dst, dpitch, P_packed, n * sizeof(float), n * sizeof(float),
                                    (size_t)wrls::packed_floats(d), hipMemcpyDeviceToDevice, s->st);
    if (e != hipSuccess) return hip_fail(e, "state import (P)");
    e = hipMemcpy2DAsync(dst + (size_t)wrls::packed_floats(d) * s->pitch, dpitch, beta,
                         n * sizeof(float), n * sizeof(float), (size_t)(3 * d),
                         hipMemcpyDeviceToDevice, s->st);
    if (e != hipSuccess) return hip_fail(e, "state import (beta)");
    s->frames = frames;
    return WRLS_OK;
}

const char *wrls_last_error(void) { return g_err; }

const char *wrls_version(void) { return "libwrls 0.1 gfx950"; }

}  // extern "C"
