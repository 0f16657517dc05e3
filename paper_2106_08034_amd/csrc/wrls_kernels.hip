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
// around memory traffic, not matrix cores.  State is stored in chunks of 64
// pixels, four entries of a pixel per 16-byte vector (wrls_internal.h), so
// that a 64-lane wavefront on a row segment moves 1 KiB of contiguous bytes
// per vector group; the bilinear gather of a uniformly moving row is then at
// most two such runs per tap row, which the L1/L2 caches merge.  Tiles are
// handed to the eight XCDs in contiguous ranges so neighbouring tiles, which
// share source rows, meet in one L2.
#include <mutex>
#include <utility>

#include "wrls_internal.h"

namespace wrls {

namespace {

constexpr int kNumXcd = 8;
// Cache policy of the streaming stores (state, output): non-temporal, so the
// written lines do not displace the gathered previous-frame state in L2.
constexpr int kStorePolicy = 2;

// Checks of the checked build (WRLS_CHECKED): expect(ok, site) is ok, and a
// false ok also raises the site's flag (a plain store of 1 from each failing
// lane).  In the shipped build it is the constant true, so the guarded
// accesses compile exactly as without it.
#ifdef WRLS_CHECKED
__device__ uint32_t g_check_flags[kNumCheckSites];
__device__ __forceinline__ bool expect(bool ok, int site)
{
    if (!ok) *(volatile uint32_t *)&g_check_flags[site] = 1u;
    return ok;
}
#else
__device__ __forceinline__ constexpr bool expect(bool, int) { return true; }
#endif

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

// Inputs, outputs and the scalar state entries go through a raw buffer
// descriptor of one whole array (built once, in scalar registers) with the
// plane or group offset as the scalar offset and a 32-bit per-lane byte
// offset.  The address needs no per-lane 64-bit math, and an access past the
// array reads 0 / is dropped instead of faulting.  The host guarantees every
// array is below 4 GiB.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9-family raw buffer, 32-bit data

__device__ __forceinline__ Rsrc array_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kRawBufferWord3);
}
__device__ __forceinline__ float bload(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(Rsrc r, uint32_t voff, uint32_t soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff,
                                          (int)soff, kStorePolicy);
}
// 16-byte accesses (four state entries of one pixel) are ordinary global
// loads and non-temporal stores of a 4-float vector: global_load_dwordx4 /
// global_store_dwordx4.  (This compiler lowers the 128-bit raw-buffer-load
// builtin to a single 32-bit load, so the buffer path is not used for them.)
// The address is the array base plus a uniform group offset plus a 32-bit
// per-pixel slot offset (vgroup, vslot).  The pointers are marked global:
// state pointers read from a device table (batched steps) would otherwise
// compile to flat accesses.
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const f4_t gcf4_t;
typedef __attribute__((address_space(1))) f4_t gf4_t;
typedef __attribute__((address_space(1))) const char gcchar_t;
typedef __attribute__((address_space(1))) char gchar_t;
// The 16-byte slot at byte offsets goff (entry group, uniform) + slot (per pixel).
__device__ __forceinline__ gcf4_t *vec_at(const float *state, uint32_t goff, uint32_t slot)
{
    return (gcf4_t *)(((gcchar_t *)state + goff) + slot);
}
__device__ __forceinline__ gf4_t *vec_at(float *state, uint32_t goff, uint32_t slot)
{
    return (gf4_t *)(((gchar_t *)state + goff) + slot);
}

// Byte offset just past pixel i's entries in a state copy of NS entries
// (the scalar remainder follows the vector groups in a chunk).
template <int NS>
__device__ __forceinline__ uint32_t pixel_end(uint32_t i)
{
    constexpr int G = vec_planes(NS);
    if constexpr (NS % 4 != 0)
        return sslot(i, NS) + sgroup(NS, NS - 4 * G - 1) + 4u;
    else
        return vslot(i, NS) + vgroup(G - 1) + 16u;
}

// Element j of plane `plane` of an input array of planes of n values.
__device__ __forceinline__ float load_in(Rsrc r, const float *, uint32_t n, int plane, uint32_t j)
{
    return bload(r, j * 4u, (uint32_t)plane * n * 4u);
}
__device__ __forceinline__ float load_in(Rsrc r, const _Float16 *, uint32_t n, int plane, uint32_t j)
{
    const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(j * 2u),
                                                           (int)((uint32_t)plane * n * 2u), 0);
    return (float)__builtin_bit_cast(_Float16, h);
}

__device__ __forceinline__ bool finite(float v) { return __builtin_isfinite(v); }

// The motion vector of pixel j (zero without a motion array); loaded ahead of
// the other inputs, since the gather's addresses wait on it.
__device__ __forceinline__ void load_motion(const FrameArgs &a, uint32_t j, uint32_t n, float &vx,
                                            float &vy)
{
    vx = 0.0f;
    vy = 0.0f;
    if (a.motion && !a.fresh) {
        const Rsrc r_mot = array_rsrc(a.motion, 2u * n * 4u);
        vx = bload(r_mot, j * 4u, 0u);
        vy = bload(r_mot, j * 4u, n * 4u);
    }
}
// Reprojection (Sec. 5.3, Table 2: pi(v_j) = j + v_j in the previous frame):
// the NS state entries of pixel (x, y) gathered from the previous frame's
// state at (x, y) + v, v = (vx, vy).  Returns false when the pixel has no
// valid source (first frame, non-finite motion, source outside the image).
// The source position is not rounded: with x an integer, floor(x + v) =
// x + floor(v), the fraction is v - floor(v), and 0 <= x + v <= W - 1 is
// -x <= v <= W - 1 - x, whose bounds are exact in binary32.  floor(v) and
// v - floor(v) are exact for v >= 0 and v <= -1; for -1 < v < 0 the fraction
// 1 + v is rounded to nearest (error <= 2^-25; 1 when |v| < 2^-25, which
// puts all the weight on the tap at x, the exact source's nearest).  A
// binary32 sum x + v would instead move the source by up to half an ulp of
// x: 1.2e-4 px near x = 3800, 4.9e-4 px past 8192.  Nearest rounds half up:
// floor(x + v + 1/2) = x + floor(v) + (fraction >= 1/2), exact since a
// rounded fraction 1 + v falls below 1/2 only where it is exact.
// The vector groups (four entries per 16-byte access) come first, then the
// scalar remainder.
template <int NS>
__device__ __forceinline__ bool gather_state(const FrameArgs &a, int x, int y, float vx, float vy,
                                             float (&st)[NS])
{
    constexpr int G = vec_planes(NS);
    if (a.fresh) return false;
    // NaN fails every comparison and +-inf lands outside: both restart.
    if (!(vx >= (float)(-x) && vx <= (float)(a.W - 1 - x) && vy >= (float)(-y) &&
          vy <= (float)(a.H - 1 - y)))
        return false;
    const float flx = floorf(vx), fly = floorf(vy);
    const float fx = vx - flx, fy = vy - fly;
    const int x0 = x + (int)flx, y0 = y + (int)fly;
    const uint32_t pitch = (uint32_t)a.pitch;
    const Rsrc src = array_rsrc(a.state_in, (uint32_t)NS * pitch * 4u);
    if (a.nearest) {
        const int xn = min(x0 + (fx >= 0.5f ? 1 : 0), a.W - 1);
        const int yn = min(y0 + (fy >= 0.5f ? 1 : 0), a.H - 1);
        const uint32_t i = (uint32_t)yn * (uint32_t)a.W + (uint32_t)xn;
        if (!expect(xn >= 0 && yn >= 0 && pixel_end<NS>(i) <= (uint32_t)NS * pitch * 4u, kChkGatherTap))
            return false;
        const uint32_t vi = vslot(i, NS);
#pragma unroll
        for (int g = 0; g < G; g++) {
            const f4_t v = *vec_at(a.state_in, vgroup(g), vi);
#pragma unroll
            for (int e = 0; e < 4; e++) st[4 * g + e] = v[e];
        }
#pragma unroll
        for (int k = 4 * G; k < NS; k++) st[k] = bload(src, sslot(i, NS), sgroup(NS, k - 4 * G));
        return true;
    }
    const int x1 = min(x0 + 1, a.W - 1), y1 = min(y0 + 1, a.H - 1);
    const uint32_t W = (uint32_t)a.W;
    const uint32_t i00 = (uint32_t)y0 * W + (uint32_t)x0, i10 = (uint32_t)y0 * W + (uint32_t)x1;
    const uint32_t i01 = (uint32_t)y1 * W + (uint32_t)x0, i11 = (uint32_t)y1 * W + (uint32_t)x1;
    if (!expect(x0 >= 0 && y0 >= 0 && x0 <= x1 && y0 <= y1 && x1 < a.W && y1 < a.H &&
                    pixel_end<NS>(i11) <= (uint32_t)NS * pitch * 4u,
                kChkGatherTap))
        return false;
    // Bilinear in nested-lerp form (exact for a constant field).  The taps
    // are issued GB vector groups at a time (4 GB 16-byte loads back to
    // back, behind a scheduling barrier, before any is consumed): one group
    // per batch up to 64 entries, two above (4K d = 10: 1109 -> 1092 us, at
    // one wave per SIMD less; d = 8 and paper mode gain nothing from two,
    // three are slower everywhere).
    const uint32_t v00 = vslot(i00, NS), v10 = vslot(i10, NS), v01 = vslot(i01, NS), v11 = vslot(i11, NS);
    constexpr int GB = NS > 64 ? 2 : 1;
#pragma unroll
    for (int g0 = 0; g0 < G; g0 += GB) {
        f4_t t[GB][4];
#pragma unroll
        for (int q = 0; q < GB; q++) {
            if (g0 + q < G) {
                const uint32_t go = vgroup(g0 + q);
                t[q][0] = *vec_at(a.state_in, go, v00);
                t[q][1] = *vec_at(a.state_in, go, v10);
                t[q][2] = *vec_at(a.state_in, go, v01);
                t[q][3] = *vec_at(a.state_in, go, v11);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < GB; q++) {
            if (g0 + q < G) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const float top = fmaf(fx, t[q][1][e] - t[q][0][e], t[q][0][e]);
                    const float bot = fmaf(fx, t[q][3][e] - t[q][2][e], t[q][2][e]);
                    st[4 * (g0 + q) + e] = fmaf(fy, bot - top, top);
                }
            }
        }
    }
    if constexpr (NS % 4 != 0) {
        constexpr int R = NS - 4 * G;
        float t00[R], t10[R], t01[R], t11[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t so = sgroup(NS, r);
            t00[r] = bload(src, sslot(i00, NS), so);
            t10[r] = bload(src, sslot(i10, NS), so);
            t01[r] = bload(src, sslot(i01, NS), so);
            t11[r] = bload(src, sslot(i11, NS), so);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < R; r++) {
            const float top = fmaf(fx, t10[r] - t00[r], t00[r]);
            const float bot = fmaf(fx, t11[r] - t01[r], t01[r]);
            st[4 * G + r] = fmaf(fy, bot - top, top);
        }
    }
    return true;
}

// The model of a pixel without history: P = I / delta (packed), beta = 0.
template <int D>
__device__ __forceinline__ void init_model(float p0, float *P, float *B)
{
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int m = i; m < D; m++) P[packed_index(D, i, m)] = (i == m) ? p0 : 0.0f;
#pragma unroll
    for (int k = 0; k < 3 * D; k++) B[k] = 0.0f;
}

// Automatic forgetting factor (the paper leaves its selection to future
// work, Sec. 7.6), after Fortescue, Kershenbaum and Ydstie (Automatica,
// 1981): lambda keeps the weighted a-posteriori error information of the
// fit at a prescribed Sigma0.  With the forgetting of Eq. 10-11 that
// information obeys V(t) = lambda V(t-1) + w sum_c e_c^2 lambda / (lambda +
// w s) (e_c the a-priori residual of Eq. 8, s = p P p^T), so V(t) = Sigma0
// is the quadratic lambda^2 + B lambda - a = 0 with a = w s and
// B = w sum_c e_c^2 / Sigma0 + a - 1.  Its positive root, in (0, 1], is
// taken in the cancellation-free form for either sign of B and limited to
// [lambda_min, lambda].  A sample without weight leaves lambda at its upper
// limit (root 1); overflow drives it to the lower one.
__device__ __forceinline__ float forgetting_factor(const FrameArgs &a, float w, float s, bool ok,
                                                   const float (&yc)[3], const float (&pred)[3])
{
    float lam = 1.0f;
    if (ok) {
        const float e0 = yc[0] - pred[0], e1 = yc[1] - pred[1], e2 = yc[2] - pred[2];
        const float ws = w * s;
        const float wb = w * fmaf(e2, e2, fmaf(e1, e1, e0 * e0));
        const float B = fmaf(wb, a.inv_sigma0, ws - 1.0f);
        const float r = sqrtf(fmaf(B, B, 4.0f * ws));
        lam = B >= 0.0f ? (2.0f * ws) / (B + r) : 0.5f * (r - B);
    }
    // fmaxf returns the limit for a NaN root (inf / inf)
    return fminf(fmaxf(lam, a.lambda_min), a.lambda);
}

// One weighted RLS update in place (Sec. 5.2-5.3) of the packed P and of B
// (3 rows of D) with predictor p, colour yc and weight w (ok: the sample is
// usable); out receives the a-posteriori prediction.  The forgetting factor
// is the frame's lambda, or chosen per pixel (forgetting_factor).
template <int D>
__device__ __forceinline__ void rls_update(float *P, float *B, const float (&p)[D],
                                           const float (&yc)[3], float w, bool ok,
                                           const FrameArgs &a, float (&out)[3])
{
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
    // a-priori predictions p beta_c^T(t-1), for the residuals of Eq. 8
    float pred[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < D; i++) acc = fmaf(p[i], B[c * D + i], acc);
        pred[c] = acc;
    }
    float lambda = a.lambda, inv_lambda = a.inv_lambda;
    if (a.auto_lambda) {
        lambda = forgetting_factor(a, w, s, ok, yc, pred);
        inv_lambda = 1.0f / lambda;
    }
    const float g = w / fmaf(w, s, lambda);

    // Residual against the previous coefficients (Eq. 8) and update (Eq. 9),
    // then the a-posteriori prediction (Eq. 6).
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const float ge = ok ? g * (yc[c] - pred[c]) : 0.0f;
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
            P[idx] = fmaf(-gki, kv[m], P[idx]) * inv_lambda;
        }
    }
}

// Stores the NS state entries of pixel j (vector groups, then the scalar
// remainder) and its output.
template <int NS>
__device__ __forceinline__ void store_pixel(const FrameArgs &a, uint32_t j, uint32_t n,
                                            const float (&st)[NS], const float (&out)[3])
{
    constexpr int G = vec_planes(NS);
    const uint32_t pitch = (uint32_t)a.pitch;
    const Rsrc dst = array_rsrc(a.state_out, (uint32_t)NS * pitch * 4u);
    const Rsrc r_out = array_rsrc(a.out, 3u * n * 4u);
    if (!expect(j < n && pixel_end<NS>(j) <= (uint32_t)NS * pitch * 4u, kChkStateStore)) return;
    const uint32_t vj = vslot(j, NS);
#pragma unroll
    for (int g = 0; g < G; g++) {
        const f4_t v = {st[4 * g], st[4 * g + 1], st[4 * g + 2], st[4 * g + 3]};
        __builtin_nontemporal_store(v, vec_at(a.state_out, vgroup(g), vj));
    }
#pragma unroll
    for (int k = 4 * G; k < NS; k++) bstore(dst, sslot(j, NS), sgroup(NS, k - 4 * G), st[k]);
#pragma unroll
    for (int c = 0; c < 3; c++) bstore(r_out, j * 4u, (uint32_t)c * n * 4u, out[c]);
}

// The per-pixel update with supplied features.  D: predictor length; InT:
// colour/feature type.  State: beta (3 rows of D), then packed P
// (D(D+1)/2 entries).
template <int D, typename InT>
__device__ __forceinline__ void update_pixel(const FrameArgs &a, int x, int y)
{
    constexpr int NS = state_floats(D);
    const uint32_t n = (uint32_t)a.W * (uint32_t)a.H;
    const uint32_t j = (uint32_t)y * (uint32_t)a.W + (uint32_t)x;
    const InT *tag = nullptr;  // selects the input type's loader
    const uint32_t in_bytes = n * (uint32_t)sizeof(InT);
    const Rsrc r_color = array_rsrc(a.color, 3u * in_bytes);
    const Rsrc r_feats = array_rsrc(a.feats, (uint32_t)(D - 1) * in_bytes);

    // Loads first, consumers after the gather, so that the inputs are in
    // flight with the motion vector and the state taps: motion (the gather
    // waits on it), predictor p = [1, features], noisy colour, variance.
    float vx, vy;
    load_motion(a, j, n, vx, vy);
    float p[D];
    p[0] = 1.0f;
#pragma unroll
    for (int i = 1; i < D; i++) p[i] = load_in(r_feats, tag, n, i - 1, j);
    float yc[3];
#pragma unroll
    for (int c = 0; c < 3; c++) yc[c] = load_in(r_color, tag, n, c, j);
    const float v = a.unit_weight ? 1.0f : bload(array_rsrc(a.var, n * 4u), j * 4u, 0u);

    float st[NS];
    if (!gather_state<NS>(a, x, y, vx, vy, st))
        init_model<D>(a.p0, st + p_entry0(D), st + beta_entry0(D));

    // Weight: inverse variance (or 1); 0 for any non-finite input.
    bool ok = finite(yc[0]) && finite(yc[1]) && finite(yc[2]);
#pragma unroll
    for (int i = 1; i < D; i++) ok = ok && finite(p[i]);
    float w;
    if (a.unit_weight) {
        w = ok ? 1.0f : 0.0f;
    } else {
        ok = ok && finite(v) && v >= 0.0f;
        w = ok ? 1.0f / fmaxf(v, a.var_floor) : 0.0f;
    }
    if (!ok) {
#pragma unroll
        for (int i = 1; i < D; i++) p[i] = finite(p[i]) ? p[i] : 0.0f;
    }
    float out[3];
    rls_update<D>(st + p_entry0(D), st + beta_entry0(D), p, yc, w, ok, a, out);
    store_pixel<NS>(a, j, n, st, out);
}

// The per-pixel update with the paper's own predictor and weight (Sec. 5.3):
// p = [1, z] with the temporal feature z of Eq. 12 and the weight of Eq. 13.
// State: beta (12), packed P (10), then the history z (3).
// col: the frame's colour over the workgroup's tile and a 1-pixel halo,
// staged in LDS as 3 planes of nc floats (NaN outside the image), rows of
// rw floats; c0: this pixel's position in a plane.
// st / have: the pixel's reprojected state and whether it has a source
// (gather_state).
constexpr int kPaperNS = state_floats(4) + 3;
__device__ __forceinline__ void update_pixel_paper(const FrameArgs &a, int x, int y,
                                                   float (&st)[kPaperNS], bool have,
                                                   const float *col, int nc, int rw, int c0)
{
    constexpr int D = 4;
    constexpr int NM = state_floats(D);  // model entries; the history follows
    constexpr int NS = kPaperNS;
    const uint32_t n = (uint32_t)a.W * (uint32_t)a.H;
    const uint32_t j = (uint32_t)y * (uint32_t)a.W + (uint32_t)x;
    (void)expect(c0 - rw - 1 >= 0 && c0 + rw + 1 < nc, kChkPaperLds);
    float yc[3];
#pragma unroll
    for (int c = 0; c < 3; c++) yc[c] = col[c * nc + c0];
    const bool ok = finite(yc[0]) && finite(yc[1]) && finite(yc[2]);

    if (!have) init_model<D>(a.p0, st + p_entry0(D), st + beta_entry0(D));
    float z[3];
    if (ok) {
        // Eq. 12: history clamped to the current colour's range over the 3x3
        // neighbourhood (inside the image, finite values), blended with the
        // current colour; without history z is the colour itself.
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (have) {
            // the halo holds NaN outside the image, so one finiteness test
            // excludes both outside and non-finite neighbours
#pragma unroll
            for (int dy = -1; dy <= 1; dy++)
#pragma unroll
                for (int dx = -1; dx <= 1; dx++)
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const float v = col[c * nc + c0 + dy * rw + dx];
                        if (finite(v)) {
                            lo[c] = fminf(lo[c], v);
                            hi[c] = fmaxf(hi[c], v);
                        }
                    }
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float psi = fminf(fmaxf(st[NM + c], lo[c]), hi[c]);
            z[c] = have ? fmaf(a.alpha, psi, (1.0f - a.alpha) * yc[c]) : yc[c];
        }
    } else {
        // no usable sample: the history is carried unchanged
#pragma unroll
        for (int c = 0; c < 3; c++) z[c] = have ? st[NM + c] : 0.0f;
    }
    float w = 0.0f;
    if (ok) {
        // Eq. 13: w = exp(-dist^2 / h^2), dist = |I - z| / (min(|I|, |z|) + eps)
        float dd = 0.0f, ny = 0.0f, nz = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float e = yc[c] - z[c];
            dd = fmaf(e, e, dd);
            ny = fmaf(yc[c], yc[c], ny);
            nz = fmaf(z[c], z[c], nz);
        }
        const float dist = sqrtf(dd) / (fminf(sqrtf(ny), sqrtf(nz)) + a.eps);
        w = expf(-(dist * dist) * a.inv_h2);
    }
    const float p[D] = {1.0f, z[0], z[1], z[2]};
    float out[3];
    rls_update<D>(st + p_entry0(D), st + beta_entry0(D), p, yc, w, ok, a, out);
#pragma unroll
    for (int c = 0; c < 3; c++) st[NM + c] = z[c];
    store_pixel<NS>(a, j, n, st, out);
}

// Tile order: the image is cut into vertical strips of strip_w tiles (the
// last strip may be narrower); tiles run strip by strip, and inside a strip
// row by row.  A tile row re-reads the bottom source rows of the tile row
// above it; narrow strips keep that reuse inside L2 (4K at d = 10: reads
// 1.14x instead of 1.48x the algorithmic bytes) but measured slower than
// the full width, which is the default -- the autotuner may pick a strip.
__device__ __forceinline__ void tile_coords(int L, int tiles_x, int tiles_y, int strip_w, int &tx,
                                            int &ty)
{
    const int n_full = tiles_x / strip_w;
    const int full = n_full * strip_w * tiles_y;
    if (L < full) {
        const int per = strip_w * tiles_y;
        const int strip = L / per;
        const int r = L - strip * per;
        ty = r / strip_w;
        tx = strip * strip_w + (r - ty * strip_w);
    } else {
        const int w_last = tiles_x - n_full * strip_w;
        const int r = L - full;
        ty = r / w_last;
        tx = n_full * strip_w + (r - ty * w_last);
    }
}

template <int D, typename InT>
__global__ void __launch_bounds__(256) step_kernel(const FrameArgs a, const TileShape ts)
{
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int tx, ty;
    tile_coords(tile, a.tiles_x, a.tiles_y, a.strip_w, tx, ty);
    const int tw_mask = (1 << ts.tw_log2) - 1;
    const int x = (tx << ts.tw_log2) + ((int)threadIdx.x & tw_mask);
    const int y = ty * (ts.block_threads >> ts.tw_log2) + ((int)threadIdx.x >> ts.tw_log2);
    if (x >= a.W || y >= a.H) return;
    update_pixel<D, InT>(a, x, y);
}

// The tile's colour and a 1-pixel halo are staged in LDS once per
// workgroup (dynamic size 3 (tw + 2) (th + 2) floats): the 3x3 clamp bounds
// then cost LDS reads instead of 27 global loads per pixel.  The colour
// loads are issued first and the state gather next, so that both are in
// flight together before the barrier.  A thread stages at most
// kPaperSlots halo pixels: (tw + 2)(th + 2) <= 3 (T + 2) <= 4 T for the
// accepted shapes (T = tw th >= 64 threads).
constexpr int kPaperSlots = 4;
template <typename InT>
__global__ void __launch_bounds__(256) paper_step_kernel(const FrameArgs a, const TileShape ts)
{
    extern __shared__ float s_col[];
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int tx, ty;
    tile_coords(tile, a.tiles_x, a.tiles_y, a.strip_w, tx, ty);
    const int tw = 1 << ts.tw_log2, th = ts.block_threads >> ts.tw_log2;
    const int lx = (int)threadIdx.x & (tw - 1), ly = (int)threadIdx.x >> ts.tw_log2;
    const int x0 = tx << ts.tw_log2, y0 = ty * th;
    const int rw = tw + 2, nc = rw * (th + 2);
    const uint32_t n = (uint32_t)a.W * (uint32_t)a.H;
    const InT *tag = nullptr;
    const Rsrc r_color = array_rsrc(a.color, 3u * n * (uint32_t)sizeof(InT));
    float cv[kPaperSlots][3];
#pragma unroll
    for (int q = 0; q < kPaperSlots; q++) {
        const int sl = (int)threadIdx.x + q * ts.block_threads;
        const int hy = sl / rw, hx = sl - hy * rw;
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy;
        const bool in = sl < nc && gx >= 0 && gx < a.W && gy >= 0 && gy < a.H;
        const uint32_t jn = in ? (uint32_t)gy * (uint32_t)a.W + (uint32_t)gx : 0u;
#pragma unroll
        for (int c = 0; c < 3; c++) cv[q][c] = in ? load_in(r_color, tag, n, c, jn) : __builtin_nanf("");
    }
    const int x = x0 + lx, y = y0 + ly;
    const bool mine = x < a.W && y < a.H;
    float st[kPaperNS];
    float vx = 0.0f, vy = 0.0f;
    if (mine) load_motion(a, (uint32_t)y * (uint32_t)a.W + (uint32_t)x, n, vx, vy);
    const bool have = mine && gather_state<kPaperNS>(a, x, y, vx, vy, st);
#pragma unroll
    for (int q = 0; q < kPaperSlots; q++) {
        const int sl = (int)threadIdx.x + q * ts.block_threads;
        if (sl < nc)
#pragma unroll
            for (int c = 0; c < 3; c++) s_col[c * nc + sl] = cv[q][c];
    }
    __syncthreads();
    if (!mine) return;  // after the barrier
    update_pixel_paper(a, x, y, st, have, s_col, nc, rw, (ly + 1) * rw + lx + 1);
}

// Initial state: P = p0 * I (p0 = 1 / delta), beta = 0 (and a zero history
// in paper mode: S = state_floats(d) + 3), every pixel.
__global__ void __launch_bounds__(256) reset_kernel(float *state, int64_t npix, int d, int S,
                                                    float p0)
{
    const int np = packed_floats(d);
    const int64_t total = (int64_t)S * npix;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / npix);
        const uint32_t j = (uint32_t)(e - (int64_t)k * npix);
        float v = 0.0f;
        if (k < np) {
            // k is a diagonal entry iff it starts a row of the packed triangle
            for (int i = 0; i < d; i++)
                if (k == packed_index(d, i, i)) v = p0;
        }
        uint32_t voff, soff;
        entry_offsets(S, d, k, j, voff, soff);
        state[(soff + voff) / 4u] = v;
    }
}

// A measurement reference for the step: its loads and stores in its tile
// order and access forms, without the reprojection and the arithmetic.  Each
// pixel loads what a step loads (motion, NF feature planes, colour, variance
// when given), reads its own NS state entries from the previous copy (no
// gather: one tap at the pixel itself), and stores them to the other copy
// with an output.  The output is a plain sum of the loaded inputs, so that no
// load is dead.  The state is moved unchanged.
template <int NS, int NF, typename InT>
__global__ void __launch_bounds__(256) probe_kernel(const FrameArgs a, const TileShape ts)
{
    constexpr int G = vec_planes(NS);
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int tx, ty;
    tile_coords(tile, a.tiles_x, a.tiles_y, a.strip_w, tx, ty);
    const int x = (tx << ts.tw_log2) + ((int)threadIdx.x & ((1 << ts.tw_log2) - 1));
    const int y = ty * (ts.block_threads >> ts.tw_log2) + ((int)threadIdx.x >> ts.tw_log2);
    if (x >= a.W || y >= a.H) return;
    const uint32_t n = (uint32_t)a.W * (uint32_t)a.H;
    const uint32_t j = (uint32_t)y * (uint32_t)a.W + (uint32_t)x;
    const InT *tag = nullptr;
    const uint32_t in_bytes = n * (uint32_t)sizeof(InT);
    float vx, vy;
    load_motion(a, j, n, vx, vy);
    float sum = vx + vy;
    if constexpr (NF > 0) {
        const Rsrc r_feats = array_rsrc(a.feats, (uint32_t)NF * in_bytes);
#pragma unroll
        for (int i = 0; i < NF; i++) sum += load_in(r_feats, tag, n, i, j);
    }
    const Rsrc r_color = array_rsrc(a.color, 3u * in_bytes);
    float out[3];
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = load_in(r_color, tag, n, c, j);
    if (a.var) sum += bload(array_rsrc(a.var, n * 4u), j * 4u, 0u);
    float st[NS];
    if (!expect(pixel_end<NS>(j) <= (uint32_t)NS * (uint32_t)a.pitch * 4u, kChkGatherTap)) return;
    const uint32_t vj = vslot(j, NS);
#pragma unroll
    for (int g = 0; g < G; g++) {
        const f4_t v = *vec_at(a.state_in, vgroup(g), vj);
#pragma unroll
        for (int e = 0; e < 4; e++) st[4 * g + e] = v[e];
    }
    const Rsrc src = array_rsrc(a.state_in, (uint32_t)NS * (uint32_t)a.pitch * 4u);
#pragma unroll
    for (int k = 4 * G; k < NS; k++) st[k] = bload(src, sslot(j, NS), sgroup(NS, k - 4 * G));
    out[0] += sum;
    store_pixel<NS>(a, j, n, st, out);
}

// Plain copy of n16 16-byte vectors, one per thread: the 16-byte loads and
// non-temporal 16-byte stores of the state accesses, without the gather.
__global__ void __launch_bounds__(256) copy_kernel(const f4_t *src, f4_t *dst, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(((gcf4_t *)src)[i], (gf4_t *)dst + i);
}

// Entries k0 .. k0 + count - 1 of every pixel between a state copy and
// caller planes [count][npix].
__global__ void __launch_bounds__(256) convert_kernel(float *state, float *planes, int64_t npix,
                                                      int d, int S, int k0, int count, int to_state)
{
    const int64_t total = (int64_t)count * npix;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / npix);
        const uint32_t j = (uint32_t)(e - (int64_t)c * npix);
        uint32_t voff, soff;
        entry_offsets(S, d, k0 + c, j, voff, soff);
        const size_t i = (soff + voff) / 4u;
        if (to_state)
            state[i] = planes[e];
        else
            planes[e] = state[i];
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
    (void)hipGetLastError();  // report this launch's error, not an older one
    b.tiles_x = tiles_x;
    b.tiles_y = tiles_y;
    const int strip_w = ts.strip_w <= 0 ? tiles_x : ts.strip_w;
    b.strip_w = strip_w > tiles_x ? tiles_x : strip_w;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block((unsigned)ts.block_threads);
    if (f16)
        hipLaunchKernelGGL((step_kernel<D, _Float16>), grid, block, 0, st, b, ts);
    else
        hipLaunchKernelGGL((step_kernel<D, float>), grid, block, 0, st, b, ts);
    return hipGetLastError();
}

// Batched step: one launch over the concatenated tiles of all frames of the
// table.  XCD k (the workgroups with blockIdx % 8 == k) owns the k-th eighth
// of the tile list, and its workgroups stride through it in lock step, so at
// any moment an XCD works on a compact window of consecutive tiles and
// vertically adjacent tiles, which share source rows, meet in one L2.  With
// a grid of 8 * ceil(tiles / 8) every workgroup takes one tile (the default:
// a finished workgroup frees its slot while its stores drain); with a
// smaller, fixed grid the kernel is persistent and its workgroups loop (on
// gfx9 a looping wave's first wait for its next loads also waits for its
// previous stores, which made that form ~20% slower on the 16-stream mix).
// The occupancy hint keeps d <= 8 at 5 waves per SIMD (96 registers, no
// spills; the per-frame kernel, without a hint, takes 104 registers and 4
// waves, and times the same with a hint of 5) except d = 7, which would
// spill at 5; d >= 9 runs at 3, as the per-frame kernel with its two-group
// gather batches.
template <int D, typename InT>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(D == 7 ? 4 : (D <= 8 ? 5 : 3))))
batch_kernel(const BatchTable *__restrict__ tab)
{
    const int G = (int)gridDim.x;
    const int xcd = (int)blockIdx.x % kNumXcd;
    const int r = (int)blockIdx.x / kNumXcd;              // rank inside the XCD
    const int on_xcd = G / kNumXcd + (xcd < G % kNumXcd);  // workgroups on this XCD
    const int total = tab->total_tiles;
    const int t0 = (int)((int64_t)total * xcd / kNumXcd);
    const int t1 = (int)((int64_t)total * (xcd + 1) / kNumXcd);
    const int tw_log2 = tab->tile.tw_log2;
    const int th = tab->tile.block_threads >> tw_log2;
    const int lx = (int)threadIdx.x & ((1 << tw_log2) - 1);
    const int ly = (int)threadIdx.x >> tw_log2;
    // frame of the first tile: count the frames that end at or before it
    // (independent scalar loads, no dependent search)
    int f = 0;
    const int n = tab->n;
    for (int k = 1; k <= kMaxBatch; k++) f += (k <= n && tab->prefix[k] <= t0 + r) ? 1 : 0;
    for (int t = t0 + r; t < t1; t += on_xcd) {
        while (expect(f < n, kChkBatchFrame) && t >= tab->prefix[f + 1]) f++;
        if (!expect(f < n, kChkBatchFrame)) break;  // a table that covers no such tile
        const FrameArgs a = tab->frame[f];
        const int local = t - tab->prefix[f];
        const int ty = local / a.tiles_x;
        const int tx = local - ty * a.tiles_x;
        const int x = (tx << tw_log2) + lx;
        const int y = ty * th + ly;
        if (x < a.W && y < a.H) update_pixel<D, InT>(a, x, y);
    }
}

template <int D>
hipError_t occupancy_batched_d(bool f16, int32_t block_threads, int *blocks_per_cu)
{
    if (f16)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            blocks_per_cu, reinterpret_cast<const void *>(&batch_kernel<D, _Float16>), block_threads, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks_per_cu, reinterpret_cast<const void *>(&batch_kernel<D, float>), block_threads, 0);
}

// Spatial blend of neighbour-model predictions (Sec. 5.3, last paragraph),
// after a step, over the current state.  Pixel i's final colour averages the
// predictions p_i beta_k^T of the models k in the 5x5 window centred on i
// (pixels inside the image) with the bilateral weight
//   w_ik = exp(-|x_k - x_i|^2 / (2 sigma_s^2) - |yhat_k - yhat_i|^2 / (2 sigma_r^2)),
// yhat being the step's output.  Since every prediction uses p_i, the sum is
// p_i (sum_k w_ik beta_k^T) / sum_k w_ik: a weighted 5x5 stencil over each of
// the 3 d beta entries, then one dot product per channel.
//
// One workgroup per 64 x kBlendTH tile; each thread computes RPT vertically
// adjacent pixels.  The guide of the tile and its 2-pixel halo is staged in
// LDS and every thread keeps its 25 RPT weights in registers.  Then the beta
// entries of the halo go through LDS one state vector group (four entries)
// at a time, in two LDS slots filled by LDS-DMA loads (no staging
// registers, no LDS stores): while the workgroup accumulates group u from
// one slot, the loads of group u + 1 fill the other, and one barrier per
// group hands it over.  The guide occupies the second slot until the weights
// are computed.  Each group's four sums are folded into their channels' dot
// products as soon as they are complete, so a thread holds 4 RPT partial
// sums rather than a whole channel's.  Halo pixels outside the image are
// never loaded: their LDS entries are zeroed once.
// A thread reads each halo row once for all RPT of its pixels (LDS reads per
// pixel: 5 (RPT + 4) / RPT per group instead of 25); every read is an
// immediate offset from one base address, and a wave's read covers 1 KB of
// consecutive bytes.  Halo reads of neighbouring tiles hit L2 (wide images
// run in vertical strips of tiles, so that a tile row's bottom rows are
// still there for the tile row below); each state entry crosses HBM about
// once.
constexpr int kBlendRW = kBlendTW + 2 * kBlendR;
constexpr int kBlendRH = kBlendTH + 2 * kBlendR;
constexpr int kBlendRN = kBlendRW * kBlendRH;
constexpr int kBlendThreads = kBlendTW * kBlendTH / kBlendRPT;
constexpr int kBlendSlots = (kBlendRN + kBlendThreads - 1) / kBlendThreads;
constexpr int kBlendK = 2 * kBlendR + 1;  // window side

// Calls f(integral_constant<int, I>) for I = 0 .. N - 1, in order.
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// 16 bytes per lane from a buffer straight into LDS (buffer_load_dwordx4
// with the lds bit): lane l of the wave writes LDS bytes lds + 16 l ..
// lds + 16 l + 15, M0 holding the wave's LDS base; lanes outside the exec
// mask write nothing.  Inline assembly, because the compiler makes every
// LDS read after such a load wait for all of them to land, a wait the blend
// places itself (wait_vm0).  The asm has no register output, and M0 is used
// by nothing else in the kernels (the compiler notes that it does not
// preserve a reserved register named as clobbered; nothing here needs it
// to).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16(Rsrc r, uint32_t lds, uint32_t voff, uint32_t soff)
{
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
                 :
                 : "s"(lds), "v"(voff), "s"(r), "s"(soff)
                 : "memory", "m0");
}
#pragma clang diagnostic pop
// Wait until no vector memory operation of this wave is in flight.
__device__ __forceinline__ void wait_vm0()
{
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // vmcnt(0); expcnt, lgkmcnt not waited on
}

// 26 KB of LDS per workgroup.  Five waves per SIMD (five workgroups per
// compute unit) where the registers fit in 96 without spilling (d <= 5,
// paper mode), else four (every d fits in 128).
template <int D, typename InT, bool PAPER>
__global__ void __launch_bounds__(kBlendThreads)
__attribute__((amdgpu_waves_per_eu(D <= 5 ? 5 : 4)))
blend_kernel(const BlendArgs a)
{
    constexpr int RPT = kBlendRPT;
    constexpr int NS = state_floats(D) + (PAPER ? 3 : 0);
    constexpr int NB = 3 * D;         // beta entries, first in the state
    constexpr int UG = (NB + 3) / 4;  // state vector groups that hold them
    static_assert(beta_entry0(D) == 0 && UG <= vec_planes(NS), "beta fills the first vector groups");
    // Two LDS slots of one state group each; the second holds the guide
    // until the weights are computed.
    __shared__ float4 s_ring[2 * kBlendRN];
    float4 *const s_guide = s_ring + kBlendRN;

    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int txi, tyi;
    tile_coords(tile, a.tiles_x, a.tiles_y, a.strip_w, txi, tyi);
    const int x0 = txi * kBlendTW, y0 = tyi * kBlendTH;
    const int tid = (int)threadIdx.x;
    const int lx = tid % kBlendTW, ly = (tid / kBlendTW) * RPT;  // first of the thread's rows
    const int x = x0 + lx;
    const uint32_t n = (uint32_t)a.W * (uint32_t)a.H;
    const uint32_t pitch = (uint32_t)a.pitch;
    const Rsrc r_state = array_rsrc(a.state, (uint32_t)NS * pitch * 4u);
    const Rsrc r_guide = array_rsrc(a.guide, 3u * n * 4u);

    // Halo slots of this thread: global pixel index, or -1 outside the image,
    // and the byte offset of the pixel's 16-byte slot in a state group.
    // Slot r of the workgroup's threads is a run of kBlendThreads consecutive
    // halo pixels, so a wave's slot r is 64 consecutive LDS entries: the
    // layout an LDS-DMA load writes.
    int hj[kBlendSlots];
    uint32_t hs[kBlendSlots];
#pragma unroll
    for (int r = 0; r < kBlendSlots; r++) {
        const int sl = tid + r * kBlendThreads;
        const int hy = sl / kBlendRW, hx = sl - hy * kBlendRW;
        const int gx = x0 - kBlendR + hx, gy = y0 - kBlendR + hy;
        const bool in = sl < kBlendRN && gx >= 0 && gx < a.W && gy >= 0 && gy < a.H;
        hj[r] = in && expect(pixel_end<NS>((uint32_t)(gy * a.W + gx)) <= (uint32_t)NS * pitch * 4u,
                             kChkBlendHalo)
                    ? gy * a.W + gx
                    : -1;
        hs[r] = vslot(hj[r] >= 0 ? (uint32_t)hj[r] : 0u, NS);
    }
    // LDS byte address of this wave's first halo slot in ring slot 0.
    const uint32_t lds_wave =
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) float4 *)s_ring +
        (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6) * 64u * 16u;
    (void)expect(ly + RPT + 2 * kBlendR <= kBlendRH && lx + 2 * kBlendR < kBlendRW, kChkBlendLds);

    // State group U of the halo goes straight into ring slot U % 2.  Halo
    // pixels outside the image keep zeros: zeroed once here in slot 0, and in
    // slot 1 by the guide's staging.
    auto issue = [&](auto uu) {
        constexpr int U = decltype(uu)::value;
#pragma unroll
        for (int r = 0; r < kBlendSlots; r++)
            if (hj[r] >= 0)
                lds_dma16(r_state, lds_wave + (uint32_t)((U % 2) * kBlendRN + r * kBlendThreads) * 16u,
                          hs[r], vgroup(U));
    };
#pragma unroll
    for (int r = 0; r < kBlendSlots; r++) {
        const int sl = tid + r * kBlendThreads;
        if (sl < kBlendRN && hj[r] < 0) s_ring[sl] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    issue(std::integral_constant<int, 0>{});

    // No early exit for pixels outside the image: every thread stages the halo.
    bool mine[RPT];
    uint32_t jr[RPT];
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        const int y = y0 + ly + r;
        mine[r] = x < a.W && y < a.H;
        jr[r] = mine[r] ? (uint32_t)y * (uint32_t)a.W + (uint32_t)x : 0u;
    }
    // entry k of pixel jj of the current state
    auto state_entry = [&](int k, uint32_t jj) {
        uint32_t voff, soff;
        entry_offsets(NS, D, k, jj, voff, soff);
        return bload(r_state, voff, soff);
    };
    // The pixels' predictors p_i, entries 1..D-1 (non-finite as 0, as in
    // the step; p_0 = 1).
    const Rsrc r_feats = array_rsrc(a.feats, (uint32_t)(D - 1) * n * (uint32_t)sizeof(InT));
    float p[RPT][D];
#pragma unroll
    for (int r = 0; r < RPT; r++)
#pragma unroll
        for (int m = 1; m < D; m++) {
            float v;
            if (PAPER) {
                v = state_entry(state_floats(D) + m - 1, jr[r]);
            } else {
                const InT *tag = nullptr;
                v = load_in(r_feats, tag, n, m - 1, jr[r]);
            }
            p[r][m] = finite(v) ? v : 0.0f;
        }

    {
        float g[kBlendSlots][3];
#pragma unroll
        for (int r = 0; r < kBlendSlots; r++)
#pragma unroll
            for (int c = 0; c < 3; c++)
                g[r][c] = hj[r] >= 0 ? bload(r_guide, (uint32_t)hj[r] * 4u, (uint32_t)c * n * 4u) : 0.0f;
#pragma unroll
        for (int r = 0; r < kBlendSlots; r++) {
            const int sl = tid + r * kBlendThreads;
            if (sl < kBlendRN) s_guide[sl] = make_float4(g[r][0], g[r][1], g[r][2], 0.0f);
        }
    }
    __syncthreads();

    // Weights: halo row hr (0 .. RPT+3 relative to the thread's first row
    // minus the radius) serves output r at row offset dy = hr - r - R.  The
    // exponent is evaluated in base 2 (exp(-e) = 2^(-e log2 e)); the spatial
    // part takes one of the five distinct squared distances 1, 2, 4, 5, 8.
    // A tile whose windows all lie inside the image (uniform over the
    // workgroup) skips the per-neighbour bounds test.
    constexpr float kLog2e = 1.4426950408889634f;
    const float nr = -a.inv2sr * kLog2e;
    float ns[9];
#pragma unroll
    for (int q = 1; q <= 8; q++) ns[q] = -(float)q * a.inv2ss * kLog2e;
    const bool interior = x0 >= kBlendR && x0 + kBlendTW + kBlendR <= a.W && y0 >= kBlendR &&
                          y0 + kBlendTH + kBlendR <= a.H;
    float4 g0[RPT];
#pragma unroll
    for (int r = 0; r < RPT; r++) g0[r] = s_guide[(ly + r + kBlendR) * kBlendRW + lx + kBlendR];
    float w[RPT][kBlendK * kBlendK];
    float den[RPT];
    auto weights = [&](auto check) {
        constexpr bool CHECK = decltype(check)::value;
#pragma unroll
        for (int r = 0; r < RPT; r++) den[r] = 1.0f;  // the centre
#pragma unroll
        for (int hr = 0; hr < RPT + 2 * kBlendR; hr++)
#pragma unroll
            for (int dx = -kBlendR; dx <= kBlendR; dx++) {
                const float4 gk = s_guide[(ly + hr) * kBlendRW + lx + kBlendR + dx];
#pragma unroll
                for (int r = 0; r < RPT; r++) {
                    const int dy = hr - r - kBlendR;
                    if (dy < -kBlendR || dy > kBlendR) continue;
                    const int idx = (dy + kBlendR) * kBlendK + (dx + kBlendR);
                    if (dx == 0 && dy == 0) {
                        w[r][idx] = 1.0f;
                        continue;
                    }
                    const float e0 = gk.x - g0[r].x, e1 = gk.y - g0[r].y, e2 = gk.z - g0[r].z;
                    const float dr2 = fmaf(e2, e2, fmaf(e1, e1, e0 * e0));
                    float wk = __builtin_amdgcn_exp2f(fmaf(dr2, nr, ns[dx * dx + dy * dy]));
                    if (CHECK) {
                        const int yy = y0 + ly + r + dy;
                        const bool in = x + dx >= 0 && x + dx < a.W && yy >= 0 && yy < a.H;
                        wk = in ? wk : 0.0f;
                    }
                    w[r][idx] = wk;
                    den[r] += wk;
                }
            }
    };
    if (interior)
        weights(std::false_type{});
    else
        weights(std::true_type{});
    float inv_den[RPT];
#pragma unroll
    for (int r = 0; r < RPT; r++) inv_den[r] = 1.0f / den[r];

    // Group 0 has landed (the predictors too: the wait takes every load),
    // and every wave is done with the guide in slot 1.
#pragma unroll
    for (int r = 0; r < RPT; r++)
#pragma unroll
        for (int m = 1; m < D; m++) asm volatile("" : : "v"(p[r][m]));
    wait_vm0();
    __syncthreads();
    float y[RPT][3];
    static_for<UG>([&](auto uu) {
        constexpr int U = decltype(uu)::value;
        if constexpr (U + 1 < UG) issue(std::integral_constant<int, U + 1>{});
        const float4 *const slot = s_ring + (U % 2) * kBlendRN;
        float acc[RPT][4];
#pragma unroll
        for (int r = 0; r < RPT; r++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[r][e] = 0.0f;
#pragma unroll
        for (int hr = 0; hr < RPT + 2 * kBlendR; hr++) {
#pragma unroll
            for (int dx = -kBlendR; dx <= kBlendR; dx++) {
                const float4 bv = slot[(ly + hr) * kBlendRW + lx + kBlendR + dx];
                const float b4[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
                for (int r = 0; r < RPT; r++) {
                    const int dy = hr - r - kBlendR;
                    if (dy < -kBlendR || dy > kBlendR) continue;
                    const float wk = w[r][(dy + kBlendR) * kBlendK + (dx + kBlendR)];
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        if (4 * U + e < NB) acc[r][e] = fmaf(wk, b4[e], acc[r][e]);
                }
            }
            // the row's products are done here, before the next row's reads
#pragma unroll
            for (int r = 0; r < RPT; r++)
#pragma unroll
                for (int e = 0; e < 4; e++)
                    if (4 * U + e < NB) asm volatile("" : "+v"(acc[r][e]));
        }
        // entry k = 4 U + e is coefficient m = k % D of channel k / D
#pragma unroll
        for (int e = 0; e < 4; e++) {
            constexpr int k0 = 4 * U;
            if (k0 + e >= NB) continue;
            const int c = (k0 + e) / D, m = (k0 + e) % D;
#pragma unroll
            for (int r = 0; r < RPT; r++) {
                y[r][c] = m == 0 ? acc[r][e] : fmaf(p[r][m], acc[r][e], y[r][c]);
                // the group's sums are complete here: otherwise the compiler
                // defers the arithmetic past the next barrier and holds
                // several groups' LDS reads at once
                asm volatile("" : "+v"(y[r][c]));
            }
        }
        if constexpr (U + 1 < UG) {
            // group U + 1 has landed, and every wave is done with slot U % 2
            __builtin_amdgcn_sched_barrier(0);
            wait_vm0();
            __syncthreads();
        }
    });
    // Stores for the pixels inside the image only.  Every value is complete
    // before the branch (an empty asm takes each one): behind a plain branch,
    // the compiler sank the whole accumulation into it and held every LDS
    // read at once.
    const Rsrc r_out = array_rsrc(a.out, 3u * n * 4u);
    float v[RPT][3];
#pragma unroll
    for (int r = 0; r < RPT; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            v[r][c] = y[r][c] * inv_den[r];
            asm volatile("" : "+v"(v[r][c]));
        }
#pragma unroll
    for (int r = 0; r < RPT; r++)
        if (mine[r])
#pragma unroll
            for (int c = 0; c < 3; c++) bstore(r_out, jr[r] * 4u, (uint32_t)c * n * 4u, v[r][c]);
}

// A part of a batched step's frame table, passed by value as a kernel
// argument (1.2 KB): frames k0 .. k0 + m - 1 and their prefix entries
// k0 .. k0 + m; the part with k0 = 0 also carries the header.
constexpr int kChunkFrames = 8;
struct TableChunk {
    int32_t k0, m;
    int32_t n, total_tiles;
    TileShape tile;
    int32_t prefix[kChunkFrames + 1];
    FrameArgs frame[kChunkFrames];
};
static_assert(sizeof(FrameArgs) % 4 == 0, "frames are copied as 32-bit words");

// Writes one part of a frame table into device memory (one workgroup,
// 32-bit words, plain global stores).
__global__ void __launch_bounds__(256) fill_table_kernel(BatchTable *tab, const TableChunk c)
{
    const uint32_t *src = reinterpret_cast<const uint32_t *>(c.frame);
    uint32_t *dst = reinterpret_cast<uint32_t *>(tab->frame + c.k0);
    const int words = c.m * (int)(sizeof(FrameArgs) / 4);
    for (int i = (int)threadIdx.x; i < words; i += (int)blockDim.x) dst[i] = src[i];
    if ((int)threadIdx.x <= c.m) tab->prefix[c.k0 + (int)threadIdx.x] = c.prefix[threadIdx.x];
    if (c.k0 == 0 && threadIdx.x == 0) {
        tab->n = c.n;
        tab->total_tiles = c.total_tiles;
        tab->tile = c.tile;
    }
}

template <int D>
hipError_t launch_blend_d(bool f16, bool paper, const BlendArgs &a, hipStream_t st)
{
    const dim3 grid((unsigned)(a.tiles_x * a.tiles_y)), block((unsigned)kBlendThreads);
    (void)hipGetLastError();  // report this launch's error, not an older one
    if constexpr (D == 4) {
        if (paper) {
            hipLaunchKernelGGL((blend_kernel<4, float, true>), grid, block, 0, st, a);
            return hipGetLastError();
        }
    }
    if (f16)
        hipLaunchKernelGGL((blend_kernel<D, _Float16, false>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((blend_kernel<D, float, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int D>
hipError_t launch_batched_d(bool f16, const BatchTable *tab, int32_t grid, int32_t block_threads,
                            hipStream_t st)
{
    (void)hipGetLastError();  // report this launch's error, not an older one
    if (f16)
        hipLaunchKernelGGL((batch_kernel<D, _Float16>), dim3((unsigned)grid),
                           dim3((unsigned)block_threads), 0, st, tab);
    else
        hipLaunchKernelGGL((batch_kernel<D, float>), dim3((unsigned)grid),
                           dim3((unsigned)block_threads), 0, st, tab);
    return hipGetLastError();
}

}  // namespace

// The frame table of steps that allocate nothing (wrls_batch_step_noalloc):
// one table per device in a fixed device array, held until the process
// ends (sizeof(BatchTable), about 9 KB).  Host code must not use the array's
// name as an address: it reaches the array through the address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current.  Every such step on a device shares the one table, so steps that
// overlap on a device race.
static __device__ __align__(256) unsigned char scratch[sizeof(BatchTable)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
BatchTable *g_scratch_ptr[kMaxDevices];
}  // namespace

#ifdef WRLS_CHECKED
// Fails the checks of the sites in mask (lane k for site k), to exercise
// the reporting path from a kernel's flag store to the host's read.
__global__ void raise_checks_kernel(uint32_t mask)
{
    const int k = (int)threadIdx.x;
    if (k < kNumCheckSites) (void)expect(((mask >> k) & 1u) == 0u, k);
}
#endif

hipError_t raise_checks(uint32_t mask, hipStream_t st)
{
#ifdef WRLS_CHECKED
    (void)hipGetLastError();
    hipLaunchKernelGGL(raise_checks_kernel, dim3(1), dim3(64), 0, st, mask);
    return hipGetLastError();
#else
    (void)mask;
    (void)st;
    return hipErrorNotSupported;
#endif
}

hipError_t read_and_clear_checks(uint32_t *flags)
{
#ifdef WRLS_CHECKED
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    e = hipMemcpyFromSymbol(flags, HIP_SYMBOL(g_check_flags), sizeof(g_check_flags));
    if (e != hipSuccess) return e;
    const uint32_t zero[kNumCheckSites] = {};
    return hipMemcpyToSymbol(HIP_SYMBOL(g_check_flags), zero, sizeof(zero));
#else
    (void)flags;
    return hipErrorNotSupported;
#endif
}

hipError_t noalloc_table(BatchTable **tab)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<BatchTable *>(ptr);
    }
    *tab = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_fill_table(BatchTable *tab, const BatchTable &host, hipStream_t st)
{
    (void)hipGetLastError();  // report this launch's error, not an older one
    for (int k0 = 0; k0 == 0 || k0 < host.n; k0 += kChunkFrames) {
        TableChunk c{};
        c.k0 = k0;
        c.m = host.n - k0 < kChunkFrames ? host.n - k0 : kChunkFrames;
        c.n = host.n;
        c.total_tiles = host.total_tiles;
        c.tile = host.tile;
        for (int i = 0; i <= c.m; i++) c.prefix[i] = host.prefix[k0 + i];
        for (int i = 0; i < c.m; i++) c.frame[i] = host.frame[k0 + i];
        hipLaunchKernelGGL(fill_table_kernel, dim3(1), dim3(256), 0, st, tab, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_reset(float *state, int64_t npix, int d, int S, float p0, hipStream_t st)
{
    (void)hipGetLastError();  // report this launch's error, not an older one
    const int64_t total = (int64_t)S * npix;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(reset_kernel, dim3((unsigned)blocks), dim3(256), 0, st, state, npix, d, S,
                       p0);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t n16, hipStream_t st)
{
    if (n16 == 0) return hipSuccess;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks > 0x7FFFFFFFu) return hipErrorInvalidValue;
    (void)hipGetLastError();
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const f4_t *>(src), static_cast<f4_t *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_convert(float *state, float *planes, int64_t npix, int d, int S, int k0,
                          int count, bool to_state, hipStream_t st)
{
    const int64_t total = (int64_t)count * npix;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    (void)hipGetLastError();
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, st, state, planes, npix,
                       d, S, k0, count, to_state ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_step_paper(bool f16, const FrameArgs &a, TileShape ts, hipStream_t st)
{
    const int tw = 1 << ts.tw_log2;
    const int th = ts.block_threads >> ts.tw_log2;
    const int tiles_x = (a.W + tw - 1) / tw;
    const int tiles_y = (a.H + th - 1) / th;
    FrameArgs b = a;
    (void)hipGetLastError();  // report this launch's error, not an older one
    b.tiles_x = tiles_x;
    b.tiles_y = tiles_y;
    const int strip_w = ts.strip_w <= 0 ? tiles_x : ts.strip_w;
    b.strip_w = strip_w > tiles_x ? tiles_x : strip_w;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block((unsigned)ts.block_threads);
    if (th < 1 || (tw + 2) * (th + 2) > kPaperSlots * ts.block_threads) return hipErrorInvalidValue;
    const size_t lds = 3u * (size_t)(tw + 2) * (size_t)(th + 2) * sizeof(float);
    if (f16)
        hipLaunchKernelGGL((paper_step_kernel<_Float16>), grid, block, lds, st, b, ts);
    else
        hipLaunchKernelGGL((paper_step_kernel<float>), grid, block, lds, st, b, ts);
    return hipGetLastError();
}

template <int NS, int NF>
hipError_t launch_probe_ns(bool f16, const FrameArgs &a, TileShape ts, hipStream_t st)
{
    const int tw = 1 << ts.tw_log2;
    const int th = ts.block_threads >> ts.tw_log2;
    FrameArgs b = a;
    b.tiles_x = (a.W + tw - 1) / tw;
    b.tiles_y = (a.H + th - 1) / th;
    const int strip_w = ts.strip_w <= 0 ? b.tiles_x : ts.strip_w;
    b.strip_w = strip_w > b.tiles_x ? b.tiles_x : strip_w;
    const dim3 grid((unsigned)(b.tiles_x * b.tiles_y)), block((unsigned)ts.block_threads);
    (void)hipGetLastError();  // report this launch's error, not an older one
    if (f16)
        hipLaunchKernelGGL((probe_kernel<NS, NF, _Float16>), grid, block, 0, st, b, ts);
    else
        hipLaunchKernelGGL((probe_kernel<NS, NF, float>), grid, block, 0, st, b, ts);
    return hipGetLastError();
}

hipError_t launch_probe(int d, bool f16, bool paper, const FrameArgs &a, TileShape ts,
                        hipStream_t st)
{
    if (paper) return d == 4 ? launch_probe_ns<kPaperNS, 0>(f16, a, ts, st) : hipErrorInvalidValue;
    switch (d) {
    case 1: return launch_probe_ns<state_floats(1), 0>(f16, a, ts, st);
    case 2: return launch_probe_ns<state_floats(2), 1>(f16, a, ts, st);
    case 3: return launch_probe_ns<state_floats(3), 2>(f16, a, ts, st);
    case 4: return launch_probe_ns<state_floats(4), 3>(f16, a, ts, st);
    case 5: return launch_probe_ns<state_floats(5), 4>(f16, a, ts, st);
    case 6: return launch_probe_ns<state_floats(6), 5>(f16, a, ts, st);
    case 7: return launch_probe_ns<state_floats(7), 6>(f16, a, ts, st);
    case 8: return launch_probe_ns<state_floats(8), 7>(f16, a, ts, st);
    case 9: return launch_probe_ns<state_floats(9), 8>(f16, a, ts, st);
    case 10: return launch_probe_ns<state_floats(10), 9>(f16, a, ts, st);
    default: return hipErrorInvalidValue;
    }
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

hipError_t launch_step_batched(int d, bool f16, const BatchTable *tab, int32_t grid,
                               int32_t block_threads, hipStream_t st)
{
    switch (d) {
    case 1: return launch_batched_d<1>(f16, tab, grid, block_threads, st);
    case 2: return launch_batched_d<2>(f16, tab, grid, block_threads, st);
    case 3: return launch_batched_d<3>(f16, tab, grid, block_threads, st);
    case 4: return launch_batched_d<4>(f16, tab, grid, block_threads, st);
    case 5: return launch_batched_d<5>(f16, tab, grid, block_threads, st);
    case 6: return launch_batched_d<6>(f16, tab, grid, block_threads, st);
    case 7: return launch_batched_d<7>(f16, tab, grid, block_threads, st);
    case 8: return launch_batched_d<8>(f16, tab, grid, block_threads, st);
    case 9: return launch_batched_d<9>(f16, tab, grid, block_threads, st);
    case 10: return launch_batched_d<10>(f16, tab, grid, block_threads, st);
    default: return hipErrorInvalidValue;
    }
}

const void *batched_kernel_fn(int d, bool f16)
{
#define WRLS_BATCH_FN(D)                                                                   \
    case D:                                                                               \
        return f16 ? reinterpret_cast<const void *>(&batch_kernel<D, _Float16>)            \
                   : reinterpret_cast<const void *>(&batch_kernel<D, float>)
    switch (d) {
        WRLS_BATCH_FN(1);
        WRLS_BATCH_FN(2);
        WRLS_BATCH_FN(3);
        WRLS_BATCH_FN(4);
        WRLS_BATCH_FN(5);
        WRLS_BATCH_FN(6);
        WRLS_BATCH_FN(7);
        WRLS_BATCH_FN(8);
        WRLS_BATCH_FN(9);
        WRLS_BATCH_FN(10);
    default: return nullptr;
    }
#undef WRLS_BATCH_FN
}

// Tiles per vertical strip of the blend's tile order.  A tile row re-reads
// the bottom two source rows of the tile row above; that reuse stays in the
// XCD's 4 MiB L2 only while a tile row's bytes (state groups, predictor
// source, guide, output) leave room for it.  Wider rows run in strips of
// about 1.25 MiB per tile row (4K at d = 10: 15 tiles; HBM reads 1.05x the
// algorithmic bytes instead of 1.46x); narrower rows run whole (1080p at
// d = 8: 2.3 MB per tile row, where strips measured 2-3% slower).
static int blend_strip_w(int d, bool f16, bool paper, int tiles_x)
{
    const int64_t px_bytes = 16 * ((3 * d + 3) / 4) + (paper ? 12 : (d - 1) * (f16 ? 2 : 4)) + 12 + 12;
    const int64_t tile_bytes = (int64_t)kBlendTW * kBlendTH * px_bytes;
    if ((int64_t)tiles_x * tile_bytes <= (int64_t)3 << 20) return tiles_x;
    const int64_t w = ((int64_t)5 << 18) / tile_bytes;
    return (int)(w < 1 ? 1 : (w > tiles_x ? tiles_x : w));
}

hipError_t launch_blend(int d, bool f16, bool paper, const BlendArgs &args, hipStream_t st)
{
    if (paper && d != 4) return hipErrorInvalidValue;
    BlendArgs a = args;
    a.strip_w = blend_strip_w(d, f16, paper, a.tiles_x);
    switch (d) {
    case 1: return launch_blend_d<1>(f16, false, a, st);
    case 2: return launch_blend_d<2>(f16, false, a, st);
    case 3: return launch_blend_d<3>(f16, false, a, st);
    case 4: return launch_blend_d<4>(f16, paper, a, st);
    case 5: return launch_blend_d<5>(f16, false, a, st);
    case 6: return launch_blend_d<6>(f16, false, a, st);
    case 7: return launch_blend_d<7>(f16, false, a, st);
    case 8: return launch_blend_d<8>(f16, false, a, st);
    case 9: return launch_blend_d<9>(f16, false, a, st);
    case 10: return launch_blend_d<10>(f16, false, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t batched_blocks_per_cu(int d, bool f16, int32_t block_threads, int *blocks_per_cu)
{
    switch (d) {
    case 1: return occupancy_batched_d<1>(f16, block_threads, blocks_per_cu);
    case 2: return occupancy_batched_d<2>(f16, block_threads, blocks_per_cu);
    case 3: return occupancy_batched_d<3>(f16, block_threads, blocks_per_cu);
    case 4: return occupancy_batched_d<4>(f16, block_threads, blocks_per_cu);
    case 5: return occupancy_batched_d<5>(f16, block_threads, blocks_per_cu);
    case 6: return occupancy_batched_d<6>(f16, block_threads, blocks_per_cu);
    case 7: return occupancy_batched_d<7>(f16, block_threads, blocks_per_cu);
    case 8: return occupancy_batched_d<8>(f16, block_threads, blocks_per_cu);
    case 9: return occupancy_batched_d<9>(f16, block_threads, blocks_per_cu);
    case 10: return occupancy_batched_d<10>(f16, block_threads, blocks_per_cu);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace wrls
