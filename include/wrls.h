/*
 * wrls.h -- C ABI of libwrls, the per-pixel weighted recursive least squares
 * (wRLS) temporal denoiser of Iglesias-Guitian, Mane and Moon, "Real-Time
 * Denoising of Volumetric Path Tracing for Direct Volume Rendering", IEEE
 * TVCG 2020 (arXiv 2106.08034), built for AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. 5, Table 2): for every frame t, given the noisy colour
 * I~(t), a per-pixel predictor p(t) and per-pixel velocities v, produce the
 * denoised colour I^(t) = p(t) beta^T(t), carrying a linear model
 * (P, beta) per pixel from frame to frame.  The model of pixel j is fetched
 * from the previous frame at pi(v_j) = j + v_j (Sec. 5.3), then updated
 * with RLS (Eq. 8, 9, 11) using the weighted gain of Eq. 14.
 *
 * Conventions shared by every call:
 *  - Images are planar and dense, row-major: a plane holds H*W values,
 *    x fastest; a [C][H][W] buffer holds C consecutive planes.
 *  - The predictor is p = [1, f_1 .. f_{d-1}]: the caller supplies the d-1
 *    feature planes, the library prepends the intercept.
 *  - Motion is backward, in pixels: (vx, vy) at pixel (x, y) says the
 *    content was at (x + vx, y + vy) in the previous frame.  Pixel centres
 *    are at integer coordinates.  A non-finite component (NaN) marks a
 *    disoccluded pixel; a source outside [0, W-1] x [0, H-1] likewise has
 *    no history.  Such pixels, and every pixel of the first frame after
 *    creation or reset, restart from P = I/delta, beta = 0.
 *  - Reprojection is bilinear on every entry of P and beta (or nearest,
 *    rounding half up).
 *  - Weight: w = 1 / max(variance, var_floor) (inverse variance), or w = 1
 *    (plain RLS, Eq. 10).  A non-finite colour, feature or variance, or a
 *    negative variance, gives w = 0: the model is carried over and only
 *    aged (P <- P / lambda, beta unchanged).
 *  - The output is the a-posteriori prediction p(t) beta^T(t) (Eq. 6).
 *  - Every pointer passed to a compute call is a DEVICE pointer on the
 *    current HIP device, owned by the caller, and must stay valid until the
 *    work enqueued on the handle's HIP stream has completed.  Calls are
 *    stream-ordered and return without synchronising.
 *  - Errors are reported by status code only; nothing aborts and no
 *    exception crosses the ABI.  wrls_last_error() returns a thread-local
 *    message for the last failing call on the calling thread.
 *  - A handle is not re-entrant: calls on one handle must not overlap
 *    (from several threads).  Distinct handles are independent.
 */
#ifndef WRLS_H
#define WRLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WRLS_OK = 0,
    WRLS_EINVAL = -1,        /* bad argument: null pointer, bad size, bad mode */
    WRLS_ENOMEM = -2,        /* device allocation failed */
    WRLS_EHIP = -3,          /* a HIP runtime call failed; text in wrls_last_error() */
    WRLS_EUNSUPPORTED = -4   /* valid request the library does not implement */
} wrls_status;

typedef enum { WRLS_F32 = 0, WRLS_F16 = 1 } wrls_dtype;

typedef enum {
    WRLS_W_INVVAR = 0,  /* w = 1 / max(variance, var_floor) */
    WRLS_W_ONE = 1,     /* w = 1: plain RLS, Eq. 10 (variance may be NULL) */
    WRLS_W_PAPER = 2    /* the paper's own predictor and weight (Sec. 5.3), d = 4:
                         * p = [1, z] with the temporal feature
                         *   z(t) = alpha Psi[z_q(t-1), I~(t)] + (1 - alpha) I~(t)  (Eq. 12),
                         * Psi clamping the reprojected history z_q per channel to
                         * the range of I~(t) over the pixel's 3x3 neighbourhood (z = I~
                         * without history), and w = exp(-dist^2 / h^2),
                         * dist = |I~ - z| / (min(|I~|, |z|) + eps)  (Eq. 13).
                         * features and variance are not used (may be NULL); the
                         * history adds 3 state entries per pixel.  The colour
                         * enters p, so p P p^T holds its square: colours above
                         * about 1e18 overflow binary32 there (the gain becomes 0). */
} wrls_weight_mode;

typedef enum { WRLS_INTERP_BILINEAR = 0, WRLS_INTERP_NEAREST = 1 } wrls_interp;

/* Largest predictor length the kernels are built for. */
#define WRLS_MAX_D 10

typedef struct {
    int32_t width, height;  /* image size in pixels, each in [1, 16384] */
    int32_t d;              /* predictor length incl. the intercept, 1..WRLS_MAX_D */
    float lambda;           /* forgetting factor in (0, 1] (Sec. 5.2, Eq. 10-11) */
    float delta;            /* prior precision > 0: P starts at I / delta */
    float var_floor;        /* smallest variance turned into a weight, >= 0 */
    int32_t in_dtype;       /* wrls_dtype of colour and features */
    int32_t weight_mode;    /* wrls_weight_mode */
    int32_t interp;         /* wrls_interp */
    float alpha;            /* WRLS_W_PAPER: history weight of Eq. 12, in [0, 1] */
    float h;                /* WRLS_W_PAPER: bandwidth of Eq. 13, > 0, 1/h^2 finite */
    float eps;              /* WRLS_W_PAPER: epsilon of Eq. 13, > 0 (finite) */
    /* Automatic forgetting factor.  The paper fixes lambda and names its
     * automatic selection as future work (Sec. 7.6).  With sigma0 > 0 the
     * library chooses it per pixel and frame by the rule of Fortescue,
     * Kershenbaum and Ydstie (Automatica 17, 1981): lambda keeps the
     * weighted a-posteriori error information of the pixel's fit at sigma0.
     * With the forgetting of Eq. 10-11 that is the positive root of
     *   lambda^2 + (b / sigma0 + a - 1) lambda - a = 0,
     *   a = w p P p^T,  b = w sum_c e_c^2  (e_c the residual of Eq. 8),
     * which lies in (0, 1], limited to [lambda_min, lambda]: the lambda
     * above becomes the upper limit.  With inverse-variance weights
     * E[b] is about 3 (1 + a), so sigma0 = 3 N sets a memory of about N
     * frames for a fitting model and forgets faster when the residuals grow
     * (an appearance change, a disocclusion the motion missed). */
    float sigma0;           /* 0: lambda fixed (default); > 0 or +inf: automatic */
    float lambda_min;       /* automatic: lower limit, in (0, lambda]; ignored when sigma0 = 0 */
} wrls_params;

typedef struct wrls_stream wrls_stream;  /* opaque, owned by the library */

/* Fills *p with defaults for a width x height image and predictor length d:
 * lambda 0.98, delta 1, var_floor 1e-6, FP32 inputs, inverse-variance
 * weights, bilinear reprojection; alpha 0.75, h 0.75, eps 1e-4 (the values
 * Sec. 5.3 and 6 use); fixed lambda (sigma0 0, lambda_min 0).  A null p is
 * ignored. */
void wrls_params_default(wrls_params *p, int32_t width, int32_t height, int32_t d);

/* Checks a parameter block without touching the GPU: WRLS_OK or
 * WRLS_EINVAL / WRLS_EUNSUPPORTED with a message.  Besides the ranges noted
 * in wrls_params, one copy of a stream's state (wrls_state_floats(d) floats
 * per pixel, pixels padded to whole 64-pixel chunks) must stay below 4 GiB: e.g. up to
 * about 17.9 Mpixel at d = 8 and 12.6 Mpixel at d = 10 (3840x2160 is 8.3). */
wrls_status wrls_params_validate(const wrls_params *p);

/* Floats of model state per pixel: d(d+1)/2 for the packed upper triangle of
 * P (Sec. 5.2: P is the d x d inverse covariance, symmetric) plus 3d for
 * beta (one coefficient row per colour channel, Sec. 5.1).  0 for a bad d.
 * WRLS_W_PAPER streams hold 3 more (the history z). */
int32_t wrls_state_floats(int32_t d);

/* Device bytes of ONE copy of the per-pixel state of a stream with these
 * parameters (the library holds two: previous and current frame).  This is
 * the figure a server admits streams by.  0 if the parameters are invalid. */
size_t wrls_state_bytes(const wrls_params *p);

/* Device bytes a stream allocates in total (both copies, padding). */
size_t wrls_stream_device_bytes(const wrls_params *p);

/* Creates a stream: allocates its state on the current HIP device and
 * enqueues its initialisation on hip_stream (a hipStream_t; NULL = the
 * default stream).  *out receives the handle.  The handle enqueues all its
 * later work on that HIP stream. */
wrls_status wrls_create_stream(const wrls_params *p, void *hip_stream, wrls_stream **out);

/* Like wrls_create_stream, but the state lives in caller-owned device
 * memory: device_mem (256-byte aligned) of at least
 * wrls_stream_device_bytes(p) bytes, which must stay valid until
 * wrls_destroy; the library never frees it.  For servers that admit streams
 * into a preallocated HBM arena without allocating per stream. */
wrls_status wrls_create_stream_in(const wrls_params *p, void *device_mem, size_t bytes,
                                  void *hip_stream, wrls_stream **out);

/* Waits for the handle's HIP stream, frees its state (unless caller-owned)
 * and the handle.  A null handle is accepted and ignored. */
wrls_status wrls_destroy(wrls_stream *s);

/* Moves the handle's later work to another HIP stream (a hipStream_t). */
wrls_status wrls_set_hip_stream(wrls_stream *s, void *hip_stream);

/* Launch shape of the per-frame kernel (the autotuner's knobs): one thread
 * per pixel, workgroups of block_threads in {64, 128, 256} threads covering a
 * tile (1 << tile_w_log2) pixels wide and block_threads >> tile_w_log2 rows
 * high; tile_w_log2 in [0, log2(block_threads)].  Tiles are processed in
 * vertical strips of strip_tiles tiles (0 = the full image width), row by row
 * inside a strip.  Results do not depend on the shape: each pixel's
 * arithmetic is the same.  Default: strip_tiles 0 and 256 x 1 (256
 * threads) when 256 divides the image width, else 128 x 1 (128 threads); in
 * paper mode (WRLS_W_PAPER) 64 x 2 (128 threads). */
wrls_status wrls_set_tile(wrls_stream *s, int32_t tile_w_log2, int32_t block_threads,
                          int32_t strip_tiles);

/* Reads back the launch shape. */
wrls_status wrls_get_tile(const wrls_stream *s, int32_t *tile_w_log2, int32_t *block_threads,
                          int32_t *strip_tiles);

/* Restarts every pixel: P = I / delta, beta = 0, frame counter 0. */
wrls_status wrls_reset(wrls_stream *s);

/* Frames processed since creation or reset (or the count passed to
 * wrls_set_state). */
int64_t wrls_frames(const wrls_stream *s);

/* One frame (Sec. 5.2-5.3).
 *   color    [3][H][W]    in_dtype   noisy colour I~(t), linear HDR
 *   features [d-1][H][W]  in_dtype   predictor entries 1..d-1 (NULL for d = 1;
 *                                    not used in WRLS_W_PAPER mode)
 *   variance [H][W]       float      per-pixel noise variance (required by
 *                                    WRLS_W_INVVAR only)
 *   motion   [2][H][W]    float      vx plane then vy plane; NULL = zero
 *   out      [3][H][W]    float      denoised colour, written
 * All are dense device arrays, aligned to their element size, caller-owned
 * and valid until the step completes on the stream; out must not overlap an
 * input (other pixels' neighbourhoods are read while outputs are written).
 * Reads the state of the previous frame and writes this frame's state.
 * WRLS_EINVAL for a missing or misaligned array, or out equal to an input. */
wrls_status wrls_step(wrls_stream *s, const void *color, const void *features,
                      const float *variance, const float *motion, float *out);

/* Copies the current state out (device pointers, stream-ordered):
 *   P_packed [d(d+1)/2][H][W]: upper triangle of P, row-major:
 *            (0,0), (0,1) .. (0,d-1), (1,1) .. (d-1,d-1);
 *   beta     [3][d][H][W]: beta[c][i] multiplies predictor entry i for
 *            colour channel c.
 * Either pointer may be NULL to skip that part. */
wrls_status wrls_get_state(const wrls_stream *s, float *P_packed, float *beta);

/* Replaces the current state (same layout, device pointers) and sets the
 * frame counter; with frames > 0 the next step reprojects from this state. */
wrls_status wrls_set_state(wrls_stream *s, const float *P_packed, const float *beta,
                           int64_t frames);

/* Spatial blend of neighbour-model predictions (Sec. 5.3, last paragraph),
 * run after wrls_step on the stream's current state.  Pixel i's final colour
 * averages, over the 5 x 5 window centred on i (pixels inside the image;
 * the window is cut at the border), the predictions p_i beta_k^T that the
 * neighbours' models make for pixel i, with the bilateral weight
 *   w_ik = exp(-|x_k - x_i|^2 / (2 sigma_s^2)) exp(-|yhat_k - yhat_i|^2 / (2 sigma_r^2)),
 * |.| Euclidean (pixels; RGB), yhat = the step's output.
 *   features  the features given to the last wrls_step ([d-1][H][W] in_dtype,
 *             device); NULL for d = 1 and in WRLS_W_PAPER mode, where
 *             p = [1, z] with the stored history.  Non-finite entries count
 *             as 0, as in the step.
 *   temporal  the output of the last wrls_step ([3][H][W] FP32, device)
 *   sigma_s   spatial width in pixels, sigma_r range width in colour units:
 *             > 0 with 1/(2 sigma^2) finite in binary32; +inf turns the
 *             factor off
 *   out       [3][H][W] FP32, device; must not overlap temporal or the
 *             features (the 5 x 5 halos are read while outputs are written)
 * Arrays are aligned to their element size.
 * Stream-ordered on the stream's HIP stream; does not change the state.
 * WRLS_EINVAL before the first step or on bad arguments. */
wrls_status wrls_blend(const wrls_stream *s, const void *features, const float *temporal,
                       float sigma_s, float sigma_r, float *out);

/* WRLS_W_PAPER streams: copies the temporal feature history z out / in
 * ([3][H][W] floats, device pointers, stream-ordered).  WRLS_EINVAL for
 * other streams. */
wrls_status wrls_get_history(const wrls_stream *s, float *z);
wrls_status wrls_set_history(wrls_stream *s, const float *z);

/* ---- Batched steps: many streams, one launch ------------------------------
 *
 * A batch advances several streams by one frame each with ONE kernel launch
 * over the concatenated tiles of all their frames.  The frames' pointers go
 * through a device-resident table that is refilled every step, so the step
 * is a HIP graph (table copy -> kernel) built once and replayed for any
 * composition of streams (up to max_streams); only the kernel node's grid
 * is updated when the tile count changes.  The grid gives each tile its own
 * workgroup by default, or is a fixed persistent grid whose workgroups loop
 * over the tiles.  Each stream's result is bitwise the same as with
 * wrls_step. */

/* Device pointers of one stream's frame; layouts as in wrls_step. */
typedef struct {
    const void *color;
    const void *features;
    const float *variance;
    const float *motion;
    float *out;
} wrls_frame;

typedef struct wrls_batch wrls_batch;  /* opaque, owned by the library */

/* Largest number of streams one batched step accepts. */
#define WRLS_MAX_BATCH 64

/* Creates a batch context for streams of predictor length d and input type
 * in_dtype, whose steps are enqueued on hip_stream (a hipStream_t; NULL:
 * the batch creates and owns a stream).  Allocates the device table (twice,
 * so one step can be prepared while the previous one runs) and pinned host
 * staging.  Streams stepped through the batch must be ordered with the
 * batch's HIP stream (create them on it, or synchronise). */
wrls_status wrls_batch_create(int32_t max_streams, int32_t d, int32_t in_dtype, void *hip_stream,
                              wrls_batch **out);

/* Waits for the batch's HIP stream and frees the batch (not the streams). */
wrls_status wrls_batch_destroy(wrls_batch *b);

/* The batch's HIP stream (a hipStream_t). */
void *wrls_batch_hip_stream(const wrls_batch *b);

/* Launch shape: tile as in wrls_set_tile, and the grid: blocks_per_cu = 0
 * (default) launches one workgroup per tile; 1..16 a persistent grid of that
 * many workgroups per compute unit; -1 a persistent grid of as many as are
 * resident at once.  Replaces the batch's graphs. */
wrls_status wrls_batch_set_tile(wrls_batch *b, int32_t tile_w_log2, int32_t block_threads,
                                int32_t blocks_per_cu);

/* 1: replay a HIP graph per step (built on first use); 0: plain enqueue
 * (copy of the table + launch).  Default 1. */
wrls_status wrls_batch_use_graph(wrls_batch *b, int32_t enable);

/* One frame for each of streams[0..n-1] (distinct handles, same d and
 * in_dtype as the batch, n <= max_streams, not WRLS_W_PAPER); frames[i]
 * belongs to streams[i].  Stream-ordered on the batch's HIP stream; returns without
 * synchronising. */
wrls_status wrls_batch_step(wrls_batch *b, int32_t n, wrls_stream *const *streams,
                            const wrls_frame *frames);

/* ---- A batched step that allocates nothing --------------------------------
 *
 * For callers that cannot allocate device memory when they step: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * wrls_batch_step keeps its frame table in device memory that
 * wrls_batch_create allocates; this variant needs no wrls_batch: the table
 * lives in a fixed array of the library, one per device (about 9 KB, held
 * until the process ends), written by small kernels whose arguments carry
 * it (no copy, no memset, no pinned staging), followed by the same batched
 * kernel with one workgroup per tile.  The call allocates nothing, on the
 * device or the host.  Streams created with wrls_create_stream_in allocate
 * nothing either.
 *
 * One frame for each of streams[0..n-1] (distinct handles with the same d
 * and input type, not WRLS_W_PAPER; 0 <= n <= WRLS_NOALLOC_MAX_STREAMS);
 * frames[i] belongs to streams[i].  tile_w_log2 and block_threads give the
 * tile as in wrls_set_tile.  Enqueued on hip_stream (a hipStream_t; NULL:
 * the null stream), which must be ordered with the streams' other work;
 * returns without synchronising.  Each stream's result is bitwise the same
 * as with wrls_step or wrls_batch_step.  Every call on a device shares that
 * device's table and it keeps the last call's contents: two calls whose
 * work overlaps on one device (on different HIP streams, or from several
 * host threads) race and must not be issued.  WRLS_EINVAL for n above the
 * maximum or a bad argument; nothing is enqueued then. */
#define WRLS_NOALLOC_MAX_STREAMS 64
wrls_status wrls_batch_step_noalloc(int32_t n, wrls_stream *const *streams, const wrls_frame *frames,
                                    int32_t tile_w_log2, int32_t block_threads, void *hip_stream);

/* The loads and stores of one wrls_step of s without the reprojection and
 * the arithmetic: a measurement reference for the step, which the benchmark
 * reports beside the HBM peak and the plain copy.  Same arguments, checks
 * and launch shape as wrls_step (Sec. 5.2-5.3 define what the step
 * computes; this computes nothing of it).  Each pixel loads its motion,
 * features, colour and variance, reads its own state entries from the
 * current copy (no gather) and writes them unchanged to the stream's other
 * copy, and writes out[c] = colour[c] (plus, in channel 0, the sum of the
 * other inputs), so the values in out mean nothing.  The stream's current
 * state and frame count are untouched: the next wrls_step proceeds as if
 * the probe had not run.  Stream-ordered; returns without synchronising.
 * WRLS_EINVAL on a bad argument. */
wrls_status wrls_traffic_probe(wrls_stream *s, const void *color, const void *features,
                               const float *variance, const float *motion, float *out);

/* Checked builds.  The library also builds as libwrls_checked.so, whose
 * kernels test every reprojection tap, every 16-byte state access and every
 * LDS index against its array before using it; a failing access is skipped
 * and its site recorded.  wrls_checked_build returns 1 in such a build and
 * 0 in the shipped one.  wrls_checked_failures synchronises the current
 * device, stores in *site_flags (if not NULL) a bit mask of the sites that
 * failed since the last call (bit 0: a gather tap, 1: a state or output
 * store, 2: a blend halo load, 3: a blend LDS index, 4: a paper-mode LDS
 * index, 5: a batched tile without a frame) and clears them; 0 means every
 * access stayed inside its array.  WRLS_EUNSUPPORTED in the shipped build,
 * WRLS_EHIP on a HIP failure.  wrls_checked_raise fails the checks of the
 * sites in site_mask from a kernel enqueued on hip_stream (NULL: the null
 * stream), so that a test can see the reporting path work end to end.  For
 * tests and debugging, not for the hot path. */
int32_t wrls_checked_build(void);
wrls_status wrls_checked_failures(uint32_t *site_flags);
wrls_status wrls_checked_raise(uint32_t site_mask, void *hip_stream);

/* Device-to-device copy of `bytes` bytes, in the state kernels' access
 * form: 16-byte loads and non-temporal 16-byte stores, one vector per
 * thread.  A utility (for example to snapshot outputs), and the read+write
 * bandwidth reference the benchmark reports beside the HBM peak.  dst and
 * src are device pointers, 16-byte aligned, not overlapping; bytes is a
 * multiple of 16 (0 is a no-op).  Stream-ordered on hip_stream (NULL: the
 * null stream); returns without synchronising.  WRLS_EINVAL on a bad
 * argument. */
wrls_status wrls_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Message of the last failing call on this thread ("" if none). */
const char *wrls_last_error(void);

/* Library version string. */
const char *wrls_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WRLS_H */
