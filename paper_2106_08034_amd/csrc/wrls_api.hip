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
    float *state[2];  // previous / current frame, S * pitch floats each (chunked layout)
    void *alloc;      // the single device allocation holding both copies
    bool owns_alloc;  // false: caller-owned memory (wrls_create_stream_in)
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

// Pixel slots of a state copy: the pixel count rounded up to an odd number
// of 64-pixel chunks, so that the two copies of a stream (placed back to
// back, 256 bytes apart) start an odd number of chunks apart.
int64_t plane_pitch(const wrls_params *p)
{
    const int64_t n = (int64_t)p->width * p->height;
    const int64_t a = (int64_t)wrls::kPlaneAlign;
    int64_t q = (n + a - 1) / a;
    if (q % 2 == 0) q += 1;
    return q * a;
}

// Default launch shapes.  Supplied features: 256 x 1 when it divides the
// width (4K d = 10: 1110 against 1129 us at 128 x 1), else 128 x 1 (a
// 1920-wide image would leave half of every row's last 256-wide tile idle).
// Paper mode: 64 x 2, since its kernel stages a colour halo per tile (fewer
// halo rows per pixel).
constexpr wrls::TileShape kDefaultTile{7, 128, 0};
constexpr wrls::TileShape kDefaultWideTile{8, 256, 0};
constexpr wrls::TileShape kDefaultPaperTile{6, 128, 0};
wrls::TileShape default_tile(const wrls_params *p)
{
    if (p->weight_mode == WRLS_W_PAPER) return kDefaultPaperTile;
    return p->width % 256 == 0 ? kDefaultWideTile : kDefaultTile;
}

bool aligned(const void *ptr, size_t bytes) { return ((uintptr_t)ptr % bytes) == 0; }

// State entries per pixel of a stream: the model, plus the history in paper mode.
int stream_state_floats(const wrls_params *p)
{
    return wrls::state_floats(p->d) + (p->weight_mode == WRLS_W_PAPER ? 3 : 0);
}

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
    p->alpha = 0.75f;
    p->h = 0.75f;
    p->eps = 1e-4f;
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
    if (p->weight_mode != WRLS_W_INVVAR && p->weight_mode != WRLS_W_ONE &&
        p->weight_mode != WRLS_W_PAPER)
        return fail(WRLS_EINVAL, "weight_mode = %d unknown", p->weight_mode);
    if (p->weight_mode == WRLS_W_PAPER) {
        if (p->d != 4) return fail(WRLS_EINVAL, "WRLS_W_PAPER needs d = 4 (p = [1, z]), got %d", p->d);
        if (!(p->alpha >= 0.0f && p->alpha <= 1.0f))
            return fail(WRLS_EINVAL, "alpha = %g outside [0, 1]", (double)p->alpha);
        // 1/h^2 must be finite in binary32, or a zero distance gives 0 * inf
        if (!(p->h > 0.0f) || !std::isfinite(p->h) || !std::isfinite(1.0f / (p->h * p->h)))
            return fail(WRLS_EINVAL, "h = %g: 1/h^2 must be finite and h > 0", (double)p->h);
        // eps > 0 keeps the distance of a black pixel whose history is black
        // defined (0 / 0 otherwise)
        if (!(p->eps > 0.0f) || !std::isfinite(p->eps))
            return fail(WRLS_EINVAL, "eps = %g must be finite and > 0", (double)p->eps);
    }
    if (p->interp != WRLS_INTERP_BILINEAR && p->interp != WRLS_INTERP_NEAREST)
        return fail(WRLS_EINVAL, "interp = %d unknown", p->interp);
    if (!(p->sigma0 >= 0.0f))
        return fail(WRLS_EINVAL, "sigma0 = %g must be >= 0 (0: fixed lambda)", (double)p->sigma0);
    if (p->sigma0 > 0.0f && !(p->lambda_min > 0.0f && p->lambda_min <= p->lambda))
        return fail(WRLS_EINVAL, "lambda_min = %g outside (0, lambda = %g]", (double)p->lambda_min,
                    (double)p->lambda);
    // The kernels address every array with 32-bit byte offsets; the state
    // copy is the largest array of a stream.
    const uint64_t copy = (uint64_t)stream_state_floats(p) * sizeof(float) *
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
    return (size_t)stream_state_floats(p) * sizeof(float) * (size_t)p->width * (size_t)p->height;
}

size_t wrls_stream_device_bytes(const wrls_params *p)
{
    if (wrls_params_validate(p) != WRLS_OK) return 0;
    // two copies, the second one 256-byte unit further on (see init_stream)
    return 2 * (size_t)stream_state_floats(p) * sizeof(float) * (size_t)plane_pitch(p) +
           wrls::kPlaneAlign * sizeof(float);
}

namespace {

// Common part of the two constructors: mem holds both state copies.
wrls_status init_stream(const wrls_params *p, void *hip_stream, void *mem, bool owns,
                        wrls_stream **out)
{
    wrls_stream *s = new (std::nothrow) wrls_stream();
    if (!s) return fail(WRLS_ENOMEM, "host allocation of the handle failed");
    s->prm = *p;
    s->st = static_cast<hipStream_t>(hip_stream);
    s->pitch = plane_pitch(p);
    s->cur = 0;
    s->frames = 0;
    s->tile = default_tile(p);
    s->alloc = mem;
    s->owns_alloc = owns;
    const size_t one = (size_t)stream_state_floats(p) * (size_t)s->pitch;
    s->state[0] = static_cast<float *>(mem);
    // the second copy starts one 256-byte unit past the end of the first,
    // so a pixel's read and write addresses are an odd number of units
    // apart (measured ~1% faster at 1080p)
    s->state[1] = s->state[0] + one + wrls::kPlaneAlign;
    const int64_t npix = (int64_t)p->width * p->height;
    hipError_t e = wrls::launch_reset(s->state[0], npix, p->d, stream_state_floats(p),
                                      1.0f / p->delta, s->st);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "state initialisation");
    }
    *out = s;
    return WRLS_OK;
}

}  // namespace

wrls_status wrls_create_stream(const wrls_params *p, void *hip_stream, wrls_stream **out)
{
    if (!out) return fail(WRLS_EINVAL, "out is NULL");
    *out = nullptr;
    wrls_status rc = wrls_params_validate(p);
    if (rc != WRLS_OK) return rc;
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, wrls_stream_device_bytes(p));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc of the stream state");
    rc = init_stream(p, hip_stream, mem, true, out);
    if (rc != WRLS_OK) (void)hipFree(mem);
    return rc;
}

wrls_status wrls_create_stream_in(const wrls_params *p, void *device_mem, size_t bytes,
                                  void *hip_stream, wrls_stream **out)
{
    if (!out) return fail(WRLS_EINVAL, "out is NULL");
    *out = nullptr;
    wrls_status rc = wrls_params_validate(p);
    if (rc != WRLS_OK) return rc;
    if (!device_mem) return fail(WRLS_EINVAL, "device_mem is NULL");
    if (((uintptr_t)device_mem & 255) != 0)
        return fail(WRLS_EINVAL, "device_mem is not 256-byte aligned");
    const size_t need = wrls_stream_device_bytes(p);
    if (bytes < need)
        return fail(WRLS_EINVAL, "device_mem holds %zu bytes, the stream needs %zu", bytes, need);
    return init_stream(p, hip_stream, device_mem, false, out);
}

wrls_status wrls_destroy(wrls_stream *s)
{
    if (!s) return WRLS_OK;
    hipError_t e1 = hipStreamSynchronize(s->st);
    hipError_t e2 = s->owns_alloc ? hipFree(s->alloc) : hipSuccess;
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
    hipError_t e = wrls::launch_reset(s->state[s->cur], npix, s->prm.d,
                                      stream_state_floats(&s->prm), 1.0f / s->prm.delta, s->st);
    if (e != hipSuccess) return hip_fail(e, "reset launch");
    s->frames = 0;
    return WRLS_OK;
}

int64_t wrls_frames(const wrls_stream *s) { return s ? s->frames : -1; }

namespace {

// Checks one frame's pointers and fills the kernel arguments of the next
// step of s (reads state[cur], writes state[1 - cur]).
wrls_status frame_args(const wrls_stream *s, const void *color, const void *features,
                       const float *variance, const float *motion, float *out,
                       wrls::FrameArgs *a)
{
    const wrls_params &p = s->prm;
    if (!color) return fail(WRLS_EINVAL, "color is NULL");
    if (!out) return fail(WRLS_EINVAL, "out is NULL");
    const bool paper = p.weight_mode == WRLS_W_PAPER;
    if (p.d > 1 && !paper && !features)
        return fail(WRLS_EINVAL, "features is NULL with d = %d", p.d);
    if (p.weight_mode == WRLS_W_INVVAR && !variance)
        return fail(WRLS_EINVAL, "variance is NULL with inverse-variance weights");
    const size_t in_size = p.in_dtype == WRLS_F16 ? 2 : 4;
    if (!aligned(color, in_size) || (features && !aligned(features, in_size)))
        return fail(WRLS_EINVAL, "color and features need %zu-byte alignment", in_size);
    if (!aligned(variance, 4) || !aligned(motion, 4) || !aligned(out, 4))
        return fail(WRLS_EINVAL, "variance, motion and out need 4-byte alignment");
    if ((const void *)out == color || (const void *)out == features ||
        (const void *)out == variance || (const void *)out == motion)
        return fail(WRLS_EINVAL, "out must not alias an input");
    *a = wrls::FrameArgs{};
    a->color = color;
    a->feats = paper ? nullptr : features;
    a->var = p.weight_mode == WRLS_W_INVVAR ? variance : nullptr;
    a->alpha = p.alpha;
    a->inv_h2 = 1.0f / (p.h * p.h);
    a->eps = p.eps;
    a->motion = motion;
    a->out = out;
    a->state_in = s->state[s->cur];
    a->state_out = s->state[1 - s->cur];
    a->W = p.width;
    a->H = p.height;
    a->pitch = s->pitch;
    a->lambda = p.lambda;
    a->inv_lambda = 1.0f / p.lambda;
    a->auto_lambda = p.sigma0 > 0.0f;
    a->inv_sigma0 = a->auto_lambda ? 1.0f / p.sigma0 : 0.0f;  // 0 for sigma0 = +inf
    a->lambda_min = a->auto_lambda ? p.lambda_min : p.lambda;
    a->p0 = 1.0f / p.delta;
    a->var_floor = p.var_floor;
    a->fresh = s->frames == 0;
    a->unit_weight = p.weight_mode == WRLS_W_ONE;
    a->nearest = p.interp == WRLS_INTERP_NEAREST;
    return WRLS_OK;
}

void advance(wrls_stream *s)
{
    s->cur = 1 - s->cur;
    s->frames++;
}

}  // namespace

wrls_status wrls_step(wrls_stream *s, const void *color, const void *features,
                      const float *variance, const float *motion, float *out)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    wrls::FrameArgs a;
    wrls_status rc = frame_args(s, color, features, variance, motion, out, &a);
    if (rc != WRLS_OK) return rc;
    const bool f16 = s->prm.in_dtype == WRLS_F16;
    hipError_t e = s->prm.weight_mode == WRLS_W_PAPER
                       ? wrls::launch_step_paper(f16, a, s->tile, s->st)
                       : wrls::launch_step(s->prm.d, f16, a, s->tile, s->st);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    advance(s);
    return WRLS_OK;
}

wrls_status wrls_traffic_probe(wrls_stream *s, const void *color, const void *features,
                               const float *variance, const float *motion, float *out)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    wrls::FrameArgs a;
    wrls_status rc = frame_args(s, color, features, variance, motion, out, &a);
    if (rc != WRLS_OK) return rc;
    a.fresh = 0;  // the motion is read as in a step with history
    hipError_t e = wrls::launch_probe(s->prm.d, s->prm.in_dtype == WRLS_F16,
                                      s->prm.weight_mode == WRLS_W_PAPER, a, s->tile, s->st);
    if (e != hipSuccess) return hip_fail(e, "probe launch");
    return WRLS_OK;  // no advance: the current state copy is untouched
}

wrls_status wrls_blend(const wrls_stream *s, const void *features, const float *temporal,
                       float sigma_s, float sigma_r, float *out)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    const wrls_params &p = s->prm;
    const bool paper = p.weight_mode == WRLS_W_PAPER;
    if (s->frames <= 0) return fail(WRLS_EINVAL, "no state yet: step a frame before blending");
    if (!temporal || !out) return fail(WRLS_EINVAL, "temporal and out are required");
    if (out == temporal) return fail(WRLS_EINVAL, "out must not alias temporal (its halo is read)");
    const size_t in_size = p.in_dtype == WRLS_F16 ? 2 : 4;
    if ((features && !aligned(features, in_size)) || !aligned(temporal, 4) || !aligned(out, 4))
        return fail(WRLS_EINVAL, "features need %zu-byte alignment, temporal and out 4-byte", in_size);
    if (p.d > 1 && !paper && !features)
        return fail(WRLS_EINVAL, "features is NULL with d = %d", p.d);
    // +inf turns a factor off (1/(2 sigma^2) = 0); 1/(2 sigma^2) must be
    // finite so that a zero distance never meets an infinite factor
    const float ss = 1.0f / (2.0f * sigma_s * sigma_s), sr = 1.0f / (2.0f * sigma_r * sigma_r);
    if (!(sigma_s > 0.0f) || !std::isfinite(ss))
        return fail(WRLS_EINVAL, "sigma_s = %g: must be > 0 with 1/(2 sigma_s^2) finite", (double)sigma_s);
    if (!(sigma_r > 0.0f) || !std::isfinite(sr))
        return fail(WRLS_EINVAL, "sigma_r = %g: must be > 0 with 1/(2 sigma_r^2) finite", (double)sigma_r);
    wrls::BlendArgs a;
    a.state = s->state[s->cur];
    a.feats = paper ? nullptr : features;
    a.guide = temporal;
    a.out = out;
    a.W = p.width;
    a.H = p.height;
    a.pitch = s->pitch;
    a.inv2ss = ss;
    a.inv2sr = sr;
    a.tiles_x = (p.width + wrls::kBlendTW - 1) / wrls::kBlendTW;
    a.tiles_y = (p.height + wrls::kBlendTH - 1) / wrls::kBlendTH;
    hipError_t e = wrls::launch_blend(p.d, p.in_dtype == WRLS_F16, paper, a, s->st);
    if (e != hipSuccess) return hip_fail(e, "blend launch");
    return WRLS_OK;
}

wrls_status wrls_get_state(const wrls_stream *s, float *P_packed, float *beta)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    const int d = s->prm.d;
    const int S = stream_state_floats(&s->prm);
    const int64_t n = (int64_t)s->prm.width * s->prm.height;
    hipError_t e;
    if (P_packed) {
        e = wrls::launch_convert(s->state[s->cur], P_packed, n, d, S, 0, wrls::packed_floats(d),
                                 false, s->st);
        if (e != hipSuccess) return hip_fail(e, "state export (P)");
    }
    if (beta) {
        e = wrls::launch_convert(s->state[s->cur], beta, n, d, S, wrls::packed_floats(d), 3 * d,
                                 false, s->st);
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
    const int S = stream_state_floats(&s->prm);
    const int64_t n = (int64_t)s->prm.width * s->prm.height;
    hipError_t e = wrls::launch_convert(s->state[s->cur], const_cast<float *>(P_packed), n,
                                        d, S, 0, wrls::packed_floats(d), true, s->st);
    if (e != hipSuccess) return hip_fail(e, "state import (P)");
    e = wrls::launch_convert(s->state[s->cur], const_cast<float *>(beta), n, d, S,
                             wrls::packed_floats(d), 3 * d, true, s->st);
    if (e != hipSuccess) return hip_fail(e, "state import (beta)");
    s->frames = frames;
    return WRLS_OK;
}

// ---- batched steps -------------------------------------------------------

struct wrls_batch {
    int32_t max_streams, d, in_dtype;
    hipStream_t st;
    bool owns_st;
    wrls::BatchTable *dev_tab[2];   // device tables, used alternately
    wrls::BatchTable *host_tab[2];  // pinned staging of each
    hipEvent_t done[2];             // recorded after the step that used slot i
    bool pending[2];
    int slot;
    wrls::TileShape tile;
    int32_t blocks_per_cu;          // 0: one workgroup per tile; > 0: persistent grid
    int32_t cu_count;
    bool use_graph;
    // per slot: graph of (table copy -> kernel); the kernel node's grid is
    // updated when the tile count changes
    hipGraph_t graph[2];            // kept alive: its node handles address the exec's nodes
    hipGraphExec_t exec[2];
    hipGraphNode_t knode[2];
    int32_t exec_grid[2];
    const wrls::BatchTable *knode_arg[2];  // storage the kernel node's argument points to
};

// C++ linkage: the helpers return HIP (C++) types
extern "C++" {
namespace {

void drop_graphs(wrls_batch *b)
{
    for (int i = 0; i < 2; i++) {
        if (b->exec[i]) {
            (void)hipGraphExecDestroy(b->exec[i]);
            b->exec[i] = nullptr;
        }
        if (b->graph[i]) {
            (void)hipGraphDestroy(b->graph[i]);
            b->graph[i] = nullptr;
        }
    }
}

// Persistent grids default to as many workgroups per CU as are resident at
// once (more would leave a tail running after the others).
hipError_t resident_blocks_per_cu(const wrls_batch *b, int32_t block_threads, int32_t *out)
{
    int n = 0;
    hipError_t e = wrls::batched_blocks_per_cu(b->d, b->in_dtype == WRLS_F16, block_threads, &n);
    if (e == hipSuccess) *out = n < 1 ? 1 : n;
    return e;
}

// Workgroups of the launch over `tiles` tiles: a multiple of 8 (one part per
// XCD), one tile each, or the fixed persistent grid.
int32_t batch_grid(const wrls_batch *b, int32_t tiles)
{
    if (b->blocks_per_cu > 0) return b->cu_count * b->blocks_per_cu;
    const int32_t g = (tiles + 7) / 8 * 8;
    return g < 8 ? 8 : g;
}

hipKernelNodeParams kernel_params(wrls_batch *b, int i, int32_t grid)
{
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(wrls::batched_kernel_fn(b->d, b->in_dtype == WRLS_F16));
    kp.gridDim = dim3((unsigned)grid);
    kp.blockDim = dim3((unsigned)b->tile.block_threads);
    kp.sharedMemBytes = 0;
    b->knode_arg[i] = b->dev_tab[i];
    static thread_local void *args[1];
    args[0] = &b->knode_arg[i];
    kp.kernelParams = args;
    kp.extra = nullptr;
    return kp;
}

// Builds slot i's graph: copy of the pinned table to the device table, then
// the batched kernel over `grid` workgroups.
hipError_t build_graph(wrls_batch *b, int i, int32_t grid)
{
    hipGraphNode_t mnode = nullptr;
    hipError_t e = hipGraphCreate(&b->graph[i], 0);
    if (e == hipSuccess)
        e = hipGraphAddMemcpyNode1D(&mnode, b->graph[i], nullptr, 0, b->dev_tab[i], b->host_tab[i],
                                    sizeof(wrls::BatchTable), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipKernelNodeParams kp = kernel_params(b, i, grid);
        e = hipGraphAddKernelNode(&b->knode[i], b->graph[i], &mnode, 1, &kp);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[i], b->graph[i], nullptr, nullptr, 0);
    if (e == hipSuccess) {
        b->exec_grid[i] = grid;
    } else {
        drop_graphs(b);
    }
    return e;
}

// Enqueues the table copy and the launch of slot i on b->st (no graph).
hipError_t enqueue_step(wrls_batch *b, int i, int32_t grid)
{
    hipError_t e = hipMemcpyAsync(b->dev_tab[i], b->host_tab[i], sizeof(wrls::BatchTable),
                                  hipMemcpyHostToDevice, b->st);
    if (e != hipSuccess) return e;
    return wrls::launch_step_batched(b->d, b->in_dtype == WRLS_F16, b->dev_tab[i], grid,
                                     b->tile.block_threads, b->st);
}

}  // namespace
}  // extern "C++"

wrls_status wrls_batch_create(int32_t max_streams, int32_t d, int32_t in_dtype, void *hip_stream,
                              wrls_batch **out)
{
    if (!out) return fail(WRLS_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_streams < 1 || max_streams > WRLS_MAX_BATCH)
        return fail(WRLS_EINVAL, "max_streams = %d outside [1, %d]", max_streams, WRLS_MAX_BATCH);
    if (d < 1 || d > WRLS_MAX_D) return fail(WRLS_EUNSUPPORTED, "d = %d outside [1, %d]", d, WRLS_MAX_D);
    if (in_dtype != WRLS_F32 && in_dtype != WRLS_F16)
        return fail(WRLS_EINVAL, "in_dtype = %d unknown", in_dtype);
    wrls_batch *b = new (std::nothrow) wrls_batch();
    if (!b) return fail(WRLS_ENOMEM, "host allocation of the batch failed");
    b->max_streams = max_streams;
    b->d = d;
    b->in_dtype = in_dtype;
    b->tile = kDefaultTile;
    b->use_graph = true;
    b->blocks_per_cu = 0;
    hipError_t e = hipSuccess;
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && !hip_stream) {
        e = hipStreamCreate(&b->st);
        b->owns_st = e == hipSuccess;
    } else {
        b->st = static_cast<hipStream_t>(hip_stream);
    }
    for (int i = 0; i < 2 && e == hipSuccess; i++) {
        e = hipMalloc(reinterpret_cast<void **>(&b->dev_tab[i]), sizeof(wrls::BatchTable));
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&b->host_tab[i]), sizeof(wrls::BatchTable),
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        wrls_status rc = hip_fail(e, "batch creation");
        wrls_batch_destroy(b);
        return rc;
    }
    *out = b;
    return WRLS_OK;
}

wrls_status wrls_batch_destroy(wrls_batch *b)
{
    if (!b) return WRLS_OK;
    hipError_t e = hipStreamSynchronize(b->st);
    drop_graphs(b);
    for (int i = 0; i < 2; i++) {
        if (b->dev_tab[i]) (void)hipFree(b->dev_tab[i]);
        if (b->host_tab[i]) (void)hipHostFree(b->host_tab[i]);
        if (b->done[i]) (void)hipEventDestroy(b->done[i]);
    }
    if (b->owns_st) (void)hipStreamDestroy(b->st);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize in batch destroy");
    return WRLS_OK;
}

void *wrls_batch_hip_stream(const wrls_batch *b) { return b ? static_cast<void *>(b->st) : nullptr; }

wrls_status wrls_batch_set_tile(wrls_batch *b, int32_t tile_w_log2, int32_t block_threads,
                                int32_t blocks_per_cu)
{
    if (!b) return fail(WRLS_EINVAL, "batch handle is NULL");
    if (block_threads != 64 && block_threads != 128 && block_threads != 256)
        return fail(WRLS_EINVAL, "block_threads = %d not in {64, 128, 256}", block_threads);
    if (tile_w_log2 < 0 || (1 << tile_w_log2) > block_threads)
        return fail(WRLS_EINVAL, "tile width 2^%d exceeds %d threads", tile_w_log2, block_threads);
    if (blocks_per_cu < -1 || blocks_per_cu > 16)
        return fail(WRLS_EINVAL, "blocks_per_cu = %d outside [-1, 16]", blocks_per_cu);
    hipError_t e = hipSuccess;
    if (blocks_per_cu == -1) {
        e = resident_blocks_per_cu(b, block_threads, &blocks_per_cu);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
    }
    e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize in batch_set_tile");
    drop_graphs(b);
    b->tile = wrls::TileShape{tile_w_log2, block_threads, 0};
    b->blocks_per_cu = blocks_per_cu;
    return WRLS_OK;
}

wrls_status wrls_batch_use_graph(wrls_batch *b, int32_t enable)
{
    if (!b) return fail(WRLS_EINVAL, "batch handle is NULL");
    b->use_graph = enable != 0;
    return WRLS_OK;
}

wrls_status wrls_batch_step(wrls_batch *b, int32_t n, wrls_stream *const *streams,
                            const wrls_frame *frames)
{
    if (!b) return fail(WRLS_EINVAL, "batch handle is NULL");
    if (n < 0 || n > b->max_streams)
        return fail(WRLS_EINVAL, "n = %d outside [0, %d]", n, b->max_streams);
    if (n > 0 && (!streams || !frames)) return fail(WRLS_EINVAL, "streams or frames is NULL");
    for (int i = 0; i < n; i++) {
        const wrls_stream *s = streams[i];
        if (!s) return fail(WRLS_EINVAL, "streams[%d] is NULL", i);
        if (s->prm.weight_mode == WRLS_W_PAPER)
            return fail(WRLS_EUNSUPPORTED, "streams[%d]: batches do not take WRLS_W_PAPER streams", i);
        if (s->prm.d != b->d || s->prm.in_dtype != b->in_dtype)
            return fail(WRLS_EINVAL, "streams[%d] has d = %d, dtype %d; the batch takes d = %d, dtype %d",
                        i, s->prm.d, s->prm.in_dtype, b->d, b->in_dtype);
        for (int k = 0; k < i; k++)
            if (streams[k] == s) return fail(WRLS_EINVAL, "stream appears twice (%d and %d)", k, i);
    }
    const int i = b->slot;
    // the staging buffer of this slot was last read by the step two calls ago
    if (b->pending[i]) {
        hipError_t e = hipEventSynchronize(b->done[i]);
        if (e != hipSuccess) return hip_fail(e, "waiting for the batch table");
        b->pending[i] = false;
    }
    wrls::BatchTable *t = b->host_tab[i];
    t->n = n;
    t->tile = b->tile;
    t->prefix[0] = 0;
    const int tw = 1 << b->tile.tw_log2;
    const int th = b->tile.block_threads >> b->tile.tw_log2;
    for (int k = 0; k < n; k++) {
        const wrls_frame &f = frames[k];
        wrls_status rc = frame_args(streams[k], f.color, f.features, f.variance, f.motion, f.out,
                                    &t->frame[k]);
        if (rc != WRLS_OK) {
            char msg[sizeof g_err];
            std::snprintf(msg, sizeof msg, "%s", g_err);
            return fail(rc, "frames[%d]: %s", k, msg);
        }
        wrls::FrameArgs &a = t->frame[k];
        a.tiles_x = (a.W + tw - 1) / tw;
        a.tiles_y = (a.H + th - 1) / th;
        a.strip_w = a.tiles_x;
        t->prefix[k + 1] = t->prefix[k] + a.tiles_x * a.tiles_y;
    }
    t->total_tiles = t->prefix[n];
    const int32_t grid = batch_grid(b, t->total_tiles);
    hipError_t e = hipSuccess;
    if (b->use_graph) {
        if (!b->exec[i]) {
            e = build_graph(b, i, grid);
            if (e != hipSuccess) return hip_fail(e, "batch graph construction");
        } else if (b->exec_grid[i] != grid) {
            hipKernelNodeParams kp = kernel_params(b, i, grid);
            e = hipGraphExecKernelNodeSetParams(b->exec[i], b->knode[i], &kp);
            if (e != hipSuccess) return hip_fail(e, "batch graph update");
            b->exec_grid[i] = grid;
        }
        e = hipGraphLaunch(b->exec[i], b->st);
    } else {
        e = enqueue_step(b, i, grid);
    }
    if (e != hipSuccess) return hip_fail(e, "batch step");
    e = hipEventRecord(b->done[i], b->st);
    if (e != hipSuccess) return hip_fail(e, "batch event");
    b->pending[i] = true;
    b->slot = 1 - i;
    for (int k = 0; k < n; k++) advance(streams[k]);
    return WRLS_OK;
}

wrls_status wrls_batch_step_noalloc(int32_t n, wrls_stream *const *streams, const wrls_frame *frames,
                                    int32_t tile_w_log2, int32_t block_threads, void *hip_stream)
{
    if (n < 0 || n > WRLS_NOALLOC_MAX_STREAMS)
        return fail(WRLS_EINVAL, "n = %d outside [0, %d]: the fixed frame table holds %d frames", n,
                    WRLS_NOALLOC_MAX_STREAMS, WRLS_NOALLOC_MAX_STREAMS);
    if (n == 0) return WRLS_OK;
    if (!streams || !frames) return fail(WRLS_EINVAL, "streams or frames is NULL");
    if (block_threads != 64 && block_threads != 128 && block_threads != 256)
        return fail(WRLS_EINVAL, "block_threads = %d not in {64, 128, 256}", block_threads);
    if (tile_w_log2 < 0 || (1 << tile_w_log2) > block_threads)
        return fail(WRLS_EINVAL, "tile width 2^%d exceeds %d threads", tile_w_log2, block_threads);
    for (int i = 0; i < n; i++) {
        const wrls_stream *s = streams[i];
        if (!s) return fail(WRLS_EINVAL, "streams[%d] is NULL", i);
        if (s->prm.weight_mode == WRLS_W_PAPER)
            return fail(WRLS_EUNSUPPORTED, "streams[%d]: batches do not take WRLS_W_PAPER streams", i);
        if (s->prm.d != streams[0]->prm.d || s->prm.in_dtype != streams[0]->prm.in_dtype)
            return fail(WRLS_EINVAL, "streams[%d] has d = %d, dtype %d; streams[0] has d = %d, dtype %d",
                        i, s->prm.d, s->prm.in_dtype, streams[0]->prm.d, streams[0]->prm.in_dtype);
        for (int k = 0; k < i; k++)
            if (streams[k] == s) return fail(WRLS_EINVAL, "stream appears twice (%d and %d)", k, i);
    }
    // the table is built on the host (no allocation: a local) and written to
    // the device's fixed table by kernels whose arguments carry it
    wrls::BatchTable t;
    t.n = n;
    t.tile = wrls::TileShape{tile_w_log2, block_threads, 0};
    t.prefix[0] = 0;
    const int tw = 1 << tile_w_log2;
    const int th = block_threads >> tile_w_log2;
    for (int k = 0; k < n; k++) {
        const wrls_frame &f = frames[k];
        wrls_status rc = frame_args(streams[k], f.color, f.features, f.variance, f.motion, f.out,
                                    &t.frame[k]);
        if (rc != WRLS_OK) {
            char msg[sizeof g_err];
            std::snprintf(msg, sizeof msg, "%s", g_err);
            return fail(rc, "frames[%d]: %s", k, msg);
        }
        wrls::FrameArgs &a = t.frame[k];
        a.tiles_x = (a.W + tw - 1) / tw;
        a.tiles_y = (a.H + th - 1) / th;
        a.strip_w = a.tiles_x;
        t.prefix[k + 1] = t.prefix[k] + a.tiles_x * a.tiles_y;
    }
    t.total_tiles = t.prefix[n];
    wrls::BatchTable *dev_tab = nullptr;
    hipError_t e = wrls::noalloc_table(&dev_tab);
    if (e != hipSuccess) return hip_fail(e, "address of the fixed frame table");
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    e = wrls::launch_fill_table(dev_tab, t, st);
    if (e != hipSuccess) return hip_fail(e, "frame table launch");
    // one workgroup per tile, a multiple of 8 (one part per XCD)
    const int32_t grid = t.total_tiles < 8 ? 8 : (t.total_tiles + 7) / 8 * 8;
    e = wrls::launch_step_batched(streams[0]->prm.d, streams[0]->prm.in_dtype == WRLS_F16, dev_tab,
                                  grid, block_threads, st);
    if (e != hipSuccess) return hip_fail(e, "batched step launch");
    for (int k = 0; k < n; k++) advance(streams[k]);
    return WRLS_OK;
}

wrls_status wrls_get_history(const wrls_stream *s, float *z)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    if (s->prm.weight_mode != WRLS_W_PAPER) return fail(WRLS_EINVAL, "the stream has no history");
    if (!z) return fail(WRLS_EINVAL, "z is NULL");
    const int64_t n = (int64_t)s->prm.width * s->prm.height;
    hipError_t e = wrls::launch_convert(s->state[s->cur], z, n, s->prm.d,
                                        stream_state_floats(&s->prm),
                                        wrls::state_floats(s->prm.d), 3, false, s->st);
    if (e != hipSuccess) return hip_fail(e, "history export");
    return WRLS_OK;
}

wrls_status wrls_set_history(wrls_stream *s, const float *z)
{
    if (!s) return fail(WRLS_EINVAL, "stream handle is NULL");
    if (s->prm.weight_mode != WRLS_W_PAPER) return fail(WRLS_EINVAL, "the stream has no history");
    if (!z) return fail(WRLS_EINVAL, "z is NULL");
    const int64_t n = (int64_t)s->prm.width * s->prm.height;
    hipError_t e = wrls::launch_convert(s->state[s->cur], const_cast<float *>(z), n, s->prm.d,
                                        stream_state_floats(&s->prm),
                                        wrls::state_floats(s->prm.d), 3, true, s->st);
    if (e != hipSuccess) return hip_fail(e, "history import");
    return WRLS_OK;
}

wrls_status wrls_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if (bytes == 0) return WRLS_OK;
    if (!dst || !src) return fail(WRLS_EINVAL, "dst and src are required");
    if (!aligned(dst, 16) || !aligned(src, 16) || bytes % 16 != 0)
        return fail(WRLS_EINVAL, "dst and src need 16-byte alignment and bytes a multiple of 16");
    const uintptr_t d0 = (uintptr_t)dst, s0 = (uintptr_t)src;
    if (d0 < s0 + bytes && s0 < d0 + bytes) return fail(WRLS_EINVAL, "dst and src overlap");
    hipError_t e = wrls::launch_copy(dst, src, bytes / 16, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return WRLS_OK;
}

wrls_status wrls_checked_failures(uint32_t *site_flags)
{
    uint32_t f[wrls::kNumCheckSites] = {};
    hipError_t e = wrls::read_and_clear_checks(f);
    if (e == hipErrorNotSupported) return fail(WRLS_EUNSUPPORTED, "this library was built without checks");
    if (e != hipSuccess) return hip_fail(e, "reading the check flags");
    uint32_t mask = 0;
    for (int i = 0; i < wrls::kNumCheckSites; i++) mask |= f[i] ? 1u << i : 0u;
    if (site_flags) *site_flags = mask;
    return WRLS_OK;
}

wrls_status wrls_checked_raise(uint32_t site_mask, void *hip_stream)
{
    hipError_t e = wrls::raise_checks(site_mask, static_cast<hipStream_t>(hip_stream));
    if (e == hipErrorNotSupported) return fail(WRLS_EUNSUPPORTED, "this library was built without checks");
    if (e != hipSuccess) return hip_fail(e, "raising check flags");
    return WRLS_OK;
}

int32_t wrls_checked_build(void)
{
#ifdef WRLS_CHECKED
    return 1;
#else
    return 0;
#endif
}

const char *wrls_last_error(void) { return g_err; }

const char *wrls_version(void) { return "libwrls 0.1 gfx950"; }

}  // extern "C"
