// HIP kernels of libwrls for gfx950 (MI355X).
//
// One thread owns one pixel and runs the whole per-frame update of the
// paper's Sec. 5.2-5.3 in registers:
//   load the noisy colour, the predictor and the variance; weight;
//   reproject the model (P, beta) from the previous frame along the motion
//   vector (bilinear gather of every state entry); gain (Eq. 14); residual
//   and coefficient update (Eq. 8-9); inverse-covariance update (Eq. 11);
//   prediction (Eq. 6); store the new state and the output.
// The work is a batch of tiny independent d x d problems: about 1.7 flop per
// byte of HBM traffic, far below the MI355X ridge, so the kernel is built
// around memory traffic, not matrix cores.  State is stored as planes (one
// plane per state entry, padded to 256 B) so that a 64-lane wavefront on a
// row segment reads and writes 256 contiguous bytes per entry; the bilinear
// gather of a uniformly moving row is then two such runs per tap row, which
// the L1/L2 caches merge.  Tiles are handed to the eight XCDs in contiguous
// ranges so neighbouring tiles, which share source rows, meet in one L2.
#include "wrls_internal.h"

namespace wrls {

namespace {

constexpr int kNumXcd = 8;

// Workgroups are dispatched to the XCDs round-robin (block b runs on XCD
// b % 8).  Map block b to a tile index so that each XCD processes one
// contiguous range of tiles: bijective on [0, nblocks).
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int per = nblocks / kNumXcd;
    const int rem = nblocks % kNumXcd;
    const int xcd = b % kNumXcd;
    const int idx = b / kNumXcd;
    const int start = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return start + idx;
}

__device__ __forceinline__ float load_in(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float load_in(const _Float16 *p, size_t i) { return (float)p[i]; }

__device__ __forceinline__ bool finite(float v) { return __builtin_isfinite(v); }

// The per-pixel update.  D: predictor length; InT: colour/feature type.
template <int D, typename InT>
__device__ __forceinline__ void update_pixel(const FrameArgs &a, int x, int y)
{
    constexpr int NP = packed_floats(D);
    constexpr int NB = 3 * D;
    const size_t n = (size_t)a.W * (size_t)a.H;
    const size_t j = (size_t)y * a.W + x;
    const InT *color = static_cast<const InT *>(a.color);
    const InT *feats = static_cast<const InT *>(a.feats);

    // Inputs: predictor p = [1, features], noisy colour, variance.
    float p[D];
    p[0] = 1.0f;
#pragma unroll
    for (int i = 1; i < D; i++) p[i] = load_in(feats, (size_t)(i - 1) * n + j);
    float yc[3];
#pragma unroll
    for (int c = 0; c < 3; c++) yc[c] = load_in(color, (size_t)c * n + j);

    // Weight: inverse variance (or 1); 0 for any non-finite input.
    bool ok = finite(yc[0]) && finite(yc[1]) && finite(yc[2]);
#pragma unroll
    for (int i = 1; i < D; i++) ok = ok && finite(p[i]);
    float w;
    if (a.unit_weight) {
        w = ok ? 1.0f : 0.0f;
    } else {
        const float v = a.var[j];
        ok = ok && finite(v) && v >= 0.0f;
        w = ok ? 1.0f / fmaxf(v, a.var_floor) : 0.0f;
    }
    if (!ok) {
#pragma unroll
        for (int i = 1; i < D; i++) p[i] = finite(p[i]) ? p[i] : 0.0f;
    }

    // Reprojection: fetch the model at j + v from the previous frame.
    float P[NP], B[NB];
    bool have = false;
    if (!a.fresh) {
        float vx = 0.0f, vy = 0.0f;
        if (a.motion) {
            vx = a.motion[j];
            vy = a.motion[n + j];
        }
        const float sx = (float)x + vx;
        const float sy = (float)y + vy;
        // NaN fails every comparison and +-inf lands outside: both restart.
        have = sx >= 0.0f && sx <= (float)(a.W - 1) && sy >= 0.0f && sy <= (float)(a.H - 1);
        if (have) {
            const float *src = a.state_in;
            const size_t pitch = (size_t)a.pitch;
            if (a.nearest) {
                const int xn = min((int)floorf(sx + 0.5f), a.W - 1);
                const int yn = min((int)floorf(sy + 0.5f), a.H - 1);
                const size_t s0 = (size_t)yn * a.W + xn;
#pragma unroll
                for (int k = 0; k < NP; k++) P[k] = src[(size_t)k * pitch + s0];
#pragma unroll
                for (int k = 0; k < NB; k++) B[k] = src[(size_t)(NP + k) * pitch + s0];
            } else {
                const float fx0 = floorf(sx), fy0 = floorf(sy);
                const float fx = sx - fx0, fy = sy - fy0;
                const int x0 = (int)fx0, y0 = (int)fy0;
                const int x1 = min(x0 + 1, a.W - 1), y1 = min(y0 + 1, a.H - 1);
                const size_t s00 = (size_t)y0 * a.W + x0, s10 = (size_t)y0 * a.W + x1;
                const size_t s01 = (size_t)y1 * a.W + x0, s11 = (size_t)y1 * a.W + x1;
                // Bilinear in nested-lerp form: exact for a constant field.
#pragma unroll
                for (int k = 0; k < NP + NB; k++) {
                    const float *pl = src + (size_t)k * pitch;
                    const float v00 = pl[s00], v10 = pl[s10], v01 = pl[s01], v11 = pl[s11];
                    const float top = fmaf(fx, v10 - v00, v00);
                    const float bot = fmaf(fx, v11 - v01, v01);
                    const float v = fmaf(fy, bot - top, top);
                    if (k < NP) P[k] = v; else B[k - NP] = v;
                }
            }
        }
    }
    if (!have) {
#pragma unroll
        for (int i = 0; i < D; i++)
#pragma unroll
            for (int m = i; m < D; m++) P[packed_index(D, i, m)] = (i == m) ? a.p0 : 0.0f;
#pragma unroll
        for (int k = 0; k < NB; k++) B[k] = 0.0f;
    }

    // Gain (Eq. 14, multiplied through by w): k = P p^T, s = p k,
    // q = g k with g = w / (lambda + w s); g = 0 when w = 0.
    float kv[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        float acc = 0.0f;
#pragma unroll
        for (int m = 0; m < D; m++)
            acc = fmaf(P[i <= m ? packed_index(D, i, m) : packed_index(D, m, i)], p[m], acc);
        kv[i] = acc;
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < D; i++) s = fmaf(p[i], kv[i], s);
    const float g = w / fmaf(w, s, a.lambda);

    // Residual against the previous coefficients (Eq. 8) and update (Eq. 9),
    // then the a-posteriori prediction (Eq. 6).
    float out[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float pred = 0.0f;
#pragma unroll
        for (int i = 0; i < D; i++) pred = fmaf(p[i], B[c * D + i], pred);
        const float ge = ok ? g * (yc[c] - pred) : 0.0f;
        float post = 0.0f;
#pragma unroll
        for (int i = 0; i < D; i++) {
            B[c * D + i] = fmaf(ge, kv[i], B[c * D + i]);
            post = fmaf(p[i], B[c * D + i], post);
        }
        out[c] = post;
    }

    // Inverse covariance (Eq. 11): P <- (P - g k k^T) / lambda on the upper
    // triangle; symmetric by construction.
#pragma unroll
    for (int i = 0; i < D; i++) {
        const float gki = g * kv[i];
#pragma unroll
        for (int m = i; m < D; m++) {
            const int idx = packed_index(D, i, m);
            P[idx] = fmaf(-gki, kv[m], P[idx]) * a.inv_lambda;
        }
    }

    float *dst = a.state_out;
    const size_t pitch = (size_t)a.pitch;
#pragma unroll
    for (int k = 0; k < NP; k++) dst[(size_t)k * pitch + j] = P[k];
#pragma unroll
    for (int k = 0; k < NB; k++) dst[(size_t)(NP + k) * pitch + j] = B[k];
#pragma unroll
    for (int c = 0; c < 3; c++) a.out[(size_t)c * n + j] = out[c];
}

template <int D, typename InT>
__global__ void __launch_bounds__(256) step_kernel(const FrameArgs a, const TileShape ts)
{
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int tw_mask = (1 << ts.tw_log2) - 1;
    const int x = (tx << ts.tw_log2) + ((int)threadIdx.x & tw_mask);
    const int y = ty * (ts.block_threads >> ts.tw_log2) + ((int)threadIdx.x >> ts.tw_log2);
    if (x >= a.W || y >= a.H) return;
    update_pixel<D, InT>(a, x, y);
}

// Initial state: P = p0 * I (p0 = 1 / delta), beta = 0, every pixel.
__global__ void __launch_bounds__(256) reset_kernel(float *state, int64_t pitch, int64_t npix,
                                                    int d, float p0)
{
    const int np = packed_floats(d);
    const int S = state_floats(d);
    const int64_t total = (int64_t)S * npix;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / npix);
        const int64_t j = e - (int64_t)k * npix;
        float v = 0.0f;
        if (k < np) {
            // k is a diagonal entry iff it starts a row of the packed triangle
            for (int i = 0; i < d; i++)
                if (k == packed_index(d, i, i)) v = p0;
        }
        state[(size_t)k * pitch + j] = v;
    }
}

template <int D>
hipError_t launch_step_d(bool f16, const FrameArgs &a, TileShape ts, hipStream_t st)
{
    const int tw = 1 << ts.tw_log2;
    const int th = ts.block_threads >> ts.tw_log2;
    const int tiles_x = (a.W + tw - 1) / tw;
    const int tiles_y = (a.H + th - 1) / th;
    FrameArgs b = a;
    b.tiles_x = tiles_x;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block((unsigned)ts.block_threads);
    if (f16)
        hipLaunchKernelGGL((step_kernel<D, _Float16>), grid, block, 0, st, b, ts);
    else
        hipLaunchKernelGGL((step_kernel<D, float>), grid, block, 0, st, b, ts);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_reset(float *state, int64_t pitch, int64_t npix, int d, float p0,
                        hipStream_t st)
{
    const int64_t total = (int64_t)state_floats(d) * npix;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(reset_kernel, dim3((unsigned)blocks), dim3(256), 0, st, state, pitch, npix,
                       d, p0);
    return hipGetLastError();
}

hipError_t launch_step(int d, bool f16, const FrameArgs &a, TileShape ts, hipStream_t st)
{
    switch (d) {
    case 1: return launch_step_d<1>(f16, a, ts, st);
    case 2: return launch_step_d<2>(f16, a, ts, st);
    case 3: return launch_step_d<3>(f16, a, ts, st);
    case 4: return launch_step_d<4>(f16, a, ts, st);
    case 5: return launch_step_d<5>(f16, a, ts, st);
    case 6: return launch_step_d<6>(f16, a, ts, st);
    case 7: return launch_step_d<7>(f16, a, ts, st);
    case 8: return launch_step_d<8>(f16, a, ts, st);
    case 9: return launch_step_d<9>(f16, a, ts, st);
    case 10: return launch_step_d<10>(f16, a, ts, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace wrls
