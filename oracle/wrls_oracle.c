/*
 * FP64 reference implementation of the per-pixel weighted recursive least
 * squares (wRLS) temporal denoiser of Iglesias-Guitian, Mane and Moon,
 * "Real-Time Denoising of Volumetric Path Tracing for Direct Volume
 * Rendering", IEEE TVCG 2020 (arXiv 2106.08034), Sec. 5.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It is plain, slow and written to be read next to the
 * paper: no blocking, no packing, no fusion.  It shares no code, header or
 * constant with the GPU library; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.
 *
 * Arithmetic: IEEE binary64, round to nearest, built without fast-math and
 * with -ffp-contract=off.  The reprojection source j + v (an integer pixel
 * coordinate plus a binary32 motion value) is evaluated without rounding:
 * the in-image test compares v with integer bounds, the tap is
 * j + floor(v) and the bilinear fraction v - floor(v).
 *
 * Per pixel j and frame t (frames counted from 0):
 *   predictor   p = [1, f_1 .. f_{d-1}]                 (Sec. 5.1, Eq. 5)
 *   weight      w = 1 / max(var, var_floor)  (inverse-variance mode)
 *               w = 1                         (plain RLS, Eq. 10)
 *               w = 0 for non-finite or negative inputs
 *   reproject   (P, beta) <- state(t-1) at q = j + v   (Sec. 5.3, Table 2 pi)
 *               bilinear (or nearest) on every entry; a pixel with no valid
 *               source (t = 0, non-finite v, q outside the image) restarts at
 *               P = I/delta, beta = 0
 *   residual    e = y - p beta^T(t-1)                   (Eq. 8)
 *   gain        q = P p^T / (lambda/w + p P p^T)        (Eq. 14; q = 0 at w = 0)
 *   coeffs      beta(t) = beta(t-1) + q e               (Eq. 9)
 *   inv. cov.   P(t) = (P - q (p P)) / lambda           (Eq. 11)
 *   output      yhat = p beta^T(t)                      (Eq. 6, a posteriori)
 * The forgetting factor is fixed, or chosen per pixel and step by the rule
 * of Fortescue, Kershenbaum and Ydstie (below; the paper leaves automatic
 * selection to future work, Sec. 7.6).
 * Colour channels share P and w and keep one beta row each (Sec. 5.1 treats
 * channels independently with the same predictor).
 *
 * Paper mode (Sec. 5.3): the predictor is the temporal feature instead of
 * supplied features, p = [1, z] (d = 4), with
 *   z(t) = alpha Psi[z_q(t-1), I~(t)] + (1 - alpha) I~(t)     (Eq. 12)
 * where z_q(t-1) is the history reprojected like the model and Psi clamps it,
 * per channel, to the range of I~(t) over the 3x3 neighbourhood of the pixel;
 * with no history z(t) = I~(t).  The weight is
 *   w = exp(-dist^2 / h^2),  dist = |I~ - z| / (min(|I~|, |z|) + eps)  (Eq. 13)
 * with Euclidean norms over the three channels.
 *
 * Spatial blend (Sec. 5.3, last paragraph), a separate pass after a step:
 * the final colour of pixel i averages, over the 5x5 window centred on i,
 * the predictions p_i beta_k^T that the neighbours' models make for pixel i,
 * with a bilateral weight (Gaussian in pixel distance times Gaussian in the
 * distance between the neighbours' temporal outputs).
 *
 * Parity pins: closed-form exponentially weighted least squares, the d = 1
 * weighted mean, brute-force stacked design matrices (Eq. 7), SPD and
 * symmetry of P, the noise-free identities, exact integer shifts and exact
 * bilinear reprojection of bilinear state fields.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_W_INVVAR 0
#define ORACLE_W_ONE 1
#define ORACLE_W_PAPER 2

#define ORACLE_INTERP_BILINEAR 0
#define ORACLE_INTERP_NEAREST 1

typedef struct oracle {
    int W, H, d;
    double lambda;     /* forgetting factor (Sec. 5.2); the upper limit of an automatic one */
    double sigma0;     /* automatic forgetting: prescribed information (0: lambda fixed) */
    double lambda_min; /* automatic forgetting: lower limit */
    double delta;      /* prior precision: P0 = I / delta */
    double var_floor;  /* smallest variance turned into a weight */
    int wmode;
    int interp;
    double alpha, h, eps;  /* paper mode: Eq. 12 history weight, Eq. 13 bandwidth and epsilon */
    long frames;       /* frames processed since creation or reset */
    /* Per-pixel state, pixel-major: P is d*d (full, row-major), beta 3*d. */
    double *P_cur, *beta_cur;
    double *P_prev, *beta_prev;
    double *z_cur, *z_prev;  /* paper mode: temporal feature history, 3 per pixel */
} oracle;

static size_t npix(const oracle *o) { return (size_t)o->W * (size_t)o->H; }

static void init_pixel(const oracle *o, double *P, double *beta)
{
    int d = o->d;
    for (int i = 0; i < d; i++)
        for (int k = 0; k < d; k++)
            P[i * d + k] = (i == k) ? 1.0 / o->delta : 0.0;
    for (int i = 0; i < 3 * d; i++) beta[i] = 0.0;
}

oracle *oracle_create(int W, int H, int d, double lambda, double delta,
                      double var_floor, int wmode, int interp)
{
    if (W <= 0 || H <= 0 || d < 1 || d > 32) return NULL;
    if (!(lambda > 0.0 && lambda <= 1.0) || !(delta > 0.0)) return NULL;
    if (wmode != ORACLE_W_INVVAR && wmode != ORACLE_W_ONE && wmode != ORACLE_W_PAPER) return NULL;
    if (wmode == ORACLE_W_PAPER && d != 4) return NULL;
    if (interp != ORACLE_INTERP_BILINEAR && interp != ORACLE_INTERP_NEAREST) return NULL;
    oracle *o = (oracle *)calloc(1, sizeof(oracle));
    if (!o) return NULL;
    o->W = W; o->H = H; o->d = d;
    o->lambda = lambda; o->delta = delta; o->var_floor = var_floor;
    o->wmode = wmode; o->interp = interp;
    o->alpha = 0.75; o->h = 0.75; o->eps = 1e-4;
    size_t n = npix(o);
    o->P_cur = (double *)malloc(n * d * d * sizeof(double));
    o->P_prev = (double *)malloc(n * d * d * sizeof(double));
    o->beta_cur = (double *)malloc(n * 3 * d * sizeof(double));
    o->beta_prev = (double *)malloc(n * 3 * d * sizeof(double));
    o->z_cur = (double *)calloc(n * 3, sizeof(double));
    o->z_prev = (double *)calloc(n * 3, sizeof(double));
    if (!o->P_cur || !o->P_prev || !o->beta_cur || !o->beta_prev || !o->z_cur || !o->z_prev) {
        free(o->P_cur); free(o->P_prev); free(o->beta_cur); free(o->beta_prev);
        free(o->z_cur); free(o->z_prev);
        free(o);
        return NULL;
    }
    for (size_t j = 0; j < n; j++)
        init_pixel(o, o->P_cur + j * d * d, o->beta_cur + j * 3 * d);
    o->frames = 0;
    return o;
}

void oracle_destroy(oracle *o)
{
    if (!o) return;
    free(o->P_cur); free(o->P_prev); free(o->beta_cur); free(o->beta_prev);
    free(o->z_cur); free(o->z_prev);
    free(o);
}

void oracle_reset(oracle *o)
{
    size_t n = npix(o);
    int d = o->d;
    for (size_t j = 0; j < n; j++)
        init_pixel(o, o->P_cur + j * d * d, o->beta_cur + j * 3 * d);
    o->frames = 0;
}

long oracle_frames(const oracle *o) { return o->frames; }

/* Paper-mode parameters: alpha of Eq. 12, h and eps of Eq. 13. */
void oracle_set_paper_params(oracle *o, double alpha, double h, double eps)
{
    o->alpha = alpha; o->h = h; o->eps = eps;
}

/* Automatic forgetting factor (see forgetting_factor): sigma0 > 0 turns it
 * on (0 turns it off), lambda_min in (0, lambda] limits it from below. */
int oracle_set_forgetting(oracle *o, double sigma0, double lambda_min)
{
    if (!(sigma0 >= 0.0)) return -1;
    if (sigma0 > 0.0 && !(lambda_min > 0.0 && lambda_min <= o->lambda)) return -1;
    o->sigma0 = sigma0;
    o->lambda_min = lambda_min;
    return 0;
}

/* Threads the per-row loop of oracle_step runs on. */
int oracle_threads(void) { return omp_get_max_threads(); }

/* Threads of the per-row loops from now on (n >= 1). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/*
 * Source of pixel coordinate j along one axis of an image n pixels long
 * (Sec. 5.3; Table 2 defines pi(v_j) = j + v_j as the pixel position in the
 * preceding frame).  Returns 0 when j + v is not in [0, n - 1] (this also
 * rejects a non-finite v).  Otherwise *i0 = floor(j + v) and *f = the
 * fraction (j + v) - floor(j + v).  Since j is an integer these are
 * j + floor(v) and v - floor(v), so nothing is rounded: the bounds j and
 * n - 1 - j are exact, floor(v) of a binary32 value is exact in binary64,
 * and so is v - floor(v) (to within 2^-54 for -1 < v < 0).  Nearest
 * (round half up) picks floor(j + v + 1/2) = j + floor(v + 1/2).
 */
static int source_axis(int j, double v, int n, int nearest, int *i0, double *f)
{
    if (!(v >= -(double)j && v <= (double)(n - 1 - j))) return 0;
    if (nearest) {
        *i0 = j + (int)floor(v + 0.5);
        *f = 0.0;
    } else {
        double fl = floor(v);
        *i0 = j + (int)fl;
        *f = v - fl;
    }
    return 1;
}

/*
 * Reprojection (Sec. 5.3): fills P, beta of pixel (x, y) from the previous
 * frame's state at (x + vx, y + vy) and returns 1, or returns 0 when the
 * pixel has no valid source (non-finite motion, source outside the image).
 */
static int reproject(const oracle *o, int x, int y, double vx, double vy,
                     double *P, double *beta)
{
    int d = o->d, W = o->W, H = o->H;
    int nearest = o->interp == ORACLE_INTERP_NEAREST;
    int x0, y0;
    double fx, fy;
    if (!source_axis(x, vx, W, nearest, &x0, &fx) || !source_axis(y, vy, H, nearest, &y0, &fy))
        return 0;

    if (nearest) {
        size_t src = (size_t)y0 * W + x0;
        memcpy(P, o->P_prev + src * d * d, sizeof(double) * d * d);
        memcpy(beta, o->beta_prev + src * 3 * d, sizeof(double) * 3 * d);
        return 1;
    }

    /* Bilinear: the four pixels around the source, each entry of P and beta
     * blended with the textbook weights.  At the last column/row the second
     * tap coincides with the first (its weight is then zero anyway). */
    int x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    double w00 = (1.0 - fx) * (1.0 - fy);
    double w10 = fx * (1.0 - fy);
    double w01 = (1.0 - fx) * fy;
    double w11 = fx * fy;
    size_t s00 = (size_t)y0 * W + x0, s10 = (size_t)y0 * W + x1;
    size_t s01 = (size_t)y1 * W + x0, s11 = (size_t)y1 * W + x1;
    for (int i = 0; i < d * d; i++)
        P[i] = w00 * o->P_prev[s00 * d * d + i] + w10 * o->P_prev[s10 * d * d + i]
             + w01 * o->P_prev[s01 * d * d + i] + w11 * o->P_prev[s11 * d * d + i];
    for (int i = 0; i < 3 * d; i++)
        beta[i] = w00 * o->beta_prev[s00 * 3 * d + i] + w10 * o->beta_prev[s10 * 3 * d + i]
                + w01 * o->beta_prev[s01 * 3 * d + i] + w11 * o->beta_prev[s11 * 3 * d + i];
    return 1;
}

/* The history z of the previous frame at the same source position, with the
 * same taps and weights as reproject() uses for the model (called only for
 * pixels that have a source). */
static void reproject_history(const oracle *o, int x, int y, double vx, double vy,
                              double *zq)
{
    int W = o->W, H = o->H;
    int nearest = o->interp == ORACLE_INTERP_NEAREST;
    int x0, y0;
    double fx, fy;
    if (!source_axis(x, vx, W, nearest, &x0, &fx) || !source_axis(y, vy, H, nearest, &y0, &fy))
        return;
    if (nearest) {
        for (int c = 0; c < 3; c++) zq[c] = o->z_prev[((size_t)y0 * W + x0) * 3 + c];
        return;
    }
    int x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    for (int c = 0; c < 3; c++)
        zq[c] = (1.0 - fx) * (1.0 - fy) * o->z_prev[((size_t)y0 * W + x0) * 3 + c]
              + fx * (1.0 - fy) * o->z_prev[((size_t)y0 * W + x1) * 3 + c]
              + (1.0 - fx) * fy * o->z_prev[((size_t)y1 * W + x0) * 3 + c]
              + fx * fy * o->z_prev[((size_t)y1 * W + x1) * 3 + c];
}

/* Temporal feature (Eq. 12).  color: the frame's planar colour; yc: this
 * pixel's colour (finite); zq: reprojected history, used when have_hist. */
static void temporal_feature(const oracle *o, const double *color, int x, int y, int have_hist,
                             const double *zq, const double *yc, double *z)
{
    int W = o->W, H = o->H;
    size_t n = npix(o);
    for (int c = 0; c < 3; c++) {
        if (!have_hist) {
            z[c] = yc[c];
            continue;
        }
        /* Psi: clamp to the range of the current colour over the 3x3
         * neighbourhood (inside the image, finite values only) */
        double lo = INFINITY, hi = -INFINITY;
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int nx = x + dx, ny = y + dy;
                if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
                double v = color[(size_t)c * n + (size_t)ny * W + nx];
                if (!isfinite(v)) continue;
                if (v < lo) lo = v;
                if (v > hi) hi = v;
            }
        double psi = zq[c] < lo ? lo : (zq[c] > hi ? hi : zq[c]);
        z[c] = o->alpha * psi + (1.0 - o->alpha) * yc[c];
    }
}

/* Weight of Eq. 13 from the colour and the temporal feature. */
static double feature_weight(const oracle *o, const double *yc, const double *z)
{
    double dd = 0.0, ny = 0.0, nz = 0.0;
    for (int c = 0; c < 3; c++) {
        dd += (yc[c] - z[c]) * (yc[c] - z[c]);
        ny += yc[c] * yc[c];
        nz += z[c] * z[c];
    }
    double dist = sqrt(dd) / (fmin(sqrt(ny), sqrt(nz)) + o->eps);
    return exp(-(dist * dist) / (o->h * o->h));
}

/* Weight of the current sample: inverse variance, or 1 for plain RLS.
 * Any non-finite input, or a negative variance, gives weight 0. */
static double sample_weight(const oracle *o, const double *y, const double *p, double var)
{
    for (int c = 0; c < 3; c++)
        if (!isfinite(y[c])) return 0.0;
    for (int i = 0; i < o->d; i++)
        if (!isfinite(p[i])) return 0.0;
    if (o->wmode == ORACLE_W_ONE) return 1.0;
    if (!isfinite(var) || var < 0.0) return 0.0;
    double v = var > o->var_floor ? var : o->var_floor;
    return 1.0 / v;
}

/*
 * Automatic forgetting factor, after Fortescue, Kershenbaum and Ydstie,
 * "Implementation of self-tuning regulators with variable forgetting
 * factors", Automatica 17 (1981): lambda is chosen at every step so that the
 * weighted a-posteriori error information of the fit stays at a prescribed
 * value Sigma0.  With the forgetting applied as in Eq. 10-11 (the old
 * information is discounted by lambda before the sample enters), that
 * information obeys V(t) = lambda V(t-1) + w sum_c e_c eps_c, where e_c is
 * the a-priori residual of channel c (Eq. 8) and eps_c = e_c lambda /
 * (lambda + w s) the a-posteriori one, s = p P p^T with the previous P.
 * Requiring V(t) = V(t-1) = Sigma0 gives
 *     (1 - lambda) (lambda + a) Sigma0 = lambda b,   a = w s,  b = w sum_c e_c^2,
 * i.e. lambda^2 + (b / Sigma0 + a - 1) lambda - a = 0, whose positive root
 * lies in (0, 1] (it is 1 when b = 0).  The root is then limited to
 * [lambda_min, lambda]: the stream's lambda is the upper limit.  A sample of
 * weight 0 carries no information: the root is 1.  sigma0 = 0 keeps lambda.
 * y: colour, pred: the a-priori predictions p beta_c^T(t-1).
 */
static double forgetting_factor(const oracle *o, double w, double s, const double *y,
                                const double *pred)
{
    if (o->sigma0 == 0.0) return o->lambda;
    double lam = 1.0;
    if (w > 0.0) {
        double e2 = 0.0;
        for (int c = 0; c < 3; c++) e2 += (y[c] - pred[c]) * (y[c] - pred[c]);
        double a = w * s, b = w * e2;
        double B = b / o->sigma0 + a - 1.0;
        lam = (-B + sqrt(B * B + 4.0 * a)) / 2.0;
    }
    if (lam > o->lambda) lam = o->lambda;
    if (lam < o->lambda_min) lam = o->lambda_min;
    return lam;
}

/*
 * One wRLS update of one pixel, in place on (P, beta).  y: noisy colour,
 * p: predictor, w: weight.  prior_out (may be NULL) receives p beta^T(t-1),
 * out receives p beta^T(t), scale_out (may be NULL) the magnitude of the
 * terms of that sum, sum_i |p_i beta_c,i(t)| (for error measures).  Returns
 * the forgetting factor of this step.
 */
static double update_pixel(const oracle *o, double *P, double *beta, const double *p,
                           const double *y, double w, double *prior_out, double *out,
                           double *scale_out)
{
    int d = o->d;
    double Ppt[32];   /* P p^T, a column */
    double pP[32];    /* p P, a row */
    double q[32];
    double pred_prior[3];

    for (int i = 0; i < d; i++) {
        double acc = 0.0;
        for (int k = 0; k < d; k++) acc += P[i * d + k] * p[k];
        Ppt[i] = acc;
    }
    for (int k = 0; k < d; k++) {
        double acc = 0.0;
        for (int i = 0; i < d; i++) acc += p[i] * P[i * d + k];
        pP[k] = acc;
    }
    double pPpt = 0.0;
    for (int i = 0; i < d; i++) pPpt += p[i] * Ppt[i];
    for (int c = 0; c < 3; c++) {
        double acc = 0.0;
        for (int i = 0; i < d; i++) acc += p[i] * beta[c * d + i];
        pred_prior[c] = acc;
    }
    double lambda = forgetting_factor(o, w, pPpt, y, pred_prior);

    /* Eq. 14.  At w = 0 the gain is its limit, zero. */
    if (w > 0.0) {
        double den = lambda / w + pPpt;
        for (int i = 0; i < d; i++) q[i] = Ppt[i] / den;
    } else {
        for (int i = 0; i < d; i++) q[i] = 0.0;
    }

    for (int c = 0; c < 3; c++) {
        double *b = beta + c * d;
        double pred = pred_prior[c];
        if (prior_out) prior_out[c] = pred;
        if (w > 0.0) {
            double e = y[c] - pred;                       /* Eq. 8 */
            for (int i = 0; i < d; i++) b[i] += q[i] * e;  /* Eq. 9 */
        }
    }

    for (int i = 0; i < d; i++)                            /* Eq. 11 */
        for (int k = 0; k < d; k++)
            P[i * d + k] = (P[i * d + k] - q[i] * pP[k]) / lambda;

    for (int c = 0; c < 3; c++) {                          /* Eq. 6 */
        double acc = 0.0, mag = 0.0;
        for (int i = 0; i < d; i++) {
            acc += p[i] * beta[c * d + i];
            mag += fabs(p[i] * beta[c * d + i]);
        }
        out[c] = acc;
        if (scale_out) scale_out[c] = mag;
    }
    return lambda;
}

/*
 * One frame.  Planar inputs, row-major planes of H*W values:
 *   color [3][H][W], feats [d-1][H][W] (may be NULL when d = 1),
 *   var [H][W] (ignored in unit-weight mode, may then be NULL),
 *   motion [2][H][W] (vx then vy, pixels, backward; may be NULL = zero).
 * out [3][H][W] receives the a-posteriori prediction, prior [3][H][W] (may be
 * NULL) the a-priori one, lam [H][W] (may be NULL) each pixel's forgetting
 * factor of this step, scale [3][H][W] (may be NULL) the magnitude of the
 * terms of the output, sum_i |p_i beta_c,i|.  Only pixels in the half-open rectangle
 * [x0, x1) x [y0, y1) are computed; elsewhere the state of this frame and the
 * outputs are left unspecified.  Returns 0, or -1 on a bad rectangle.
 */
int oracle_step(oracle *o, const double *color, const double *feats, const double *var,
                const double *motion, double *out, double *prior, double *lam,
                double *scale, int x0, int y0, int x1, int y1)
{
    int W = o->W, H = o->H, d = o->d;
    if (x0 < 0 || y0 < 0 || x1 > W || y1 > H || x0 > x1 || y0 > y1) return -1;
    size_t n = npix(o);

    /* The state of the previous frame becomes the source of this frame. */
    double *t;
    t = o->P_prev; o->P_prev = o->P_cur; o->P_cur = t;
    t = o->beta_prev; o->beta_prev = o->beta_cur; o->beta_cur = t;
    t = o->z_prev; o->z_prev = o->z_cur; o->z_cur = t;
    long frame = o->frames;
    int paper = o->wmode == ORACLE_W_PAPER;

#pragma omp parallel for schedule(dynamic, 1)
    for (int y = y0; y < y1; y++) {
        for (int x = x0; x < x1; x++) {
            size_t j = (size_t)y * W + x;
            double *P = o->P_cur + j * d * d;
            double *beta = o->beta_cur + j * 3 * d;
            double p[32], yc[3], o3[3], pr3[3], sc3[3];

            for (int c = 0; c < 3; c++) yc[c] = color[(size_t)c * n + j];
            int have = 0;
            double vx = motion ? motion[j] : 0.0;
            double vy = motion ? motion[n + j] : 0.0;
            if (frame > 0) have = reproject(o, x, y, vx, vy, P, beta);
            if (!have) init_pixel(o, P, beta);

            double w;
            p[0] = 1.0;
            if (paper) {
                double zq[3] = {0.0, 0.0, 0.0}, z[3];
                if (have) reproject_history(o, x, y, vx, vy, zq);
                if (isfinite(yc[0]) && isfinite(yc[1]) && isfinite(yc[2])) {
                    temporal_feature(o, color, x, y, have, zq, yc, z);
                    w = feature_weight(o, yc, z);
                } else {
                    /* no usable sample: the history is carried unchanged */
                    for (int c = 0; c < 3; c++) z[c] = zq[c];
                    w = 0.0;
                }
                for (int c = 0; c < 3; c++) {
                    p[1 + c] = z[c];
                    o->z_cur[j * 3 + c] = z[c];
                }
            } else {
                for (int i = 1; i < d; i++) p[i] = feats[(size_t)(i - 1) * n + j];
                double v = var ? var[j] : 1.0;
                w = sample_weight(o, yc, p, v);
                if (w == 0.0)  /* keep non-finite predictor entries out of P */
                    for (int i = 0; i < d; i++)
                        if (!isfinite(p[i])) p[i] = 0.0;
            }

            double lam_j = update_pixel(o, P, beta, p, yc, w, pr3, o3, sc3);
            if (lam) lam[j] = lam_j;
            for (int c = 0; c < 3; c++) {
                out[(size_t)c * n + j] = o3[c];
                if (prior) prior[(size_t)c * n + j] = pr3[c];
                if (scale) scale[(size_t)c * n + j] = sc3[c];
            }
        }
    }
    o->frames = frame + 1;
    return 0;
}

/* State export, planar: P [d][d][H][W] (full matrix), beta [3][d][H][W]. */
void oracle_get_state(const oracle *o, double *P, double *beta)
{
    size_t n = npix(o);
    int d = o->d;
    for (size_t j = 0; j < n; j++) {
        for (int i = 0; i < d * d; i++) P[(size_t)i * n + j] = o->P_cur[j * d * d + i];
        for (int i = 0; i < 3 * d; i++) beta[(size_t)i * n + j] = o->beta_cur[j * 3 * d + i];
    }
}

/* Paper mode: the temporal feature history, planar [3][H][W]. */
void oracle_get_history(const oracle *o, double *z)
{
    size_t n = npix(o);
    for (size_t j = 0; j < n; j++)
        for (int c = 0; c < 3; c++) z[(size_t)c * n + j] = o->z_cur[j * 3 + c];
}

void oracle_set_history(oracle *o, const double *z)
{
    size_t n = npix(o);
    for (size_t j = 0; j < n; j++)
        for (int c = 0; c < 3; c++) o->z_cur[j * 3 + c] = z[(size_t)c * n + j];
}

/* beta alone, planar [3][d][H][W]. */
void oracle_get_beta(const oracle *o, double *beta)
{
    size_t n = npix(o);
    int d = o->d;
    for (size_t j = 0; j < n; j++)
        for (int i = 0; i < 3 * d; i++) beta[(size_t)i * n + j] = o->beta_cur[j * 3 * d + i];
}

/* State import (same layout).  The next step reprojects from it. */
void oracle_set_state(oracle *o, const double *P, const double *beta, long frames)
{
    size_t n = npix(o);
    int d = o->d;
    for (size_t j = 0; j < n; j++) {
        for (int i = 0; i < d * d; i++) o->P_cur[j * d * d + i] = P[(size_t)i * n + j];
        for (int i = 0; i < 3 * d; i++) o->beta_cur[j * 3 * d + i] = beta[(size_t)i * n + j];
    }
    o->frames = frames;
}

/* The predictor of pixel j for the blend: [1, features] or, in paper mode,
 * [1, z] with the stored history.  Non-finite entries enter as 0, as they
 * do in the step's output. */
static void blend_predictor(const oracle *o, const double *feats, size_t j, double *p)
{
    size_t n = npix(o);
    p[0] = 1.0;
    for (int i = 1; i < o->d; i++) {
        double v = o->wmode == ORACLE_W_PAPER ? o->z_cur[j * 3 + (size_t)(i - 1)]
                                              : feats[(size_t)(i - 1) * n + j];
        p[i] = isfinite(v) ? v : 0.0;
    }
}

/*
 * Spatial blend of neighbour-model predictions (Sec. 5.3, last paragraph)
 * on the current state.  For each pixel i, over the pixels k of the 5x5
 * window centred on i that lie inside the image:
 *   out_i = sum_k w_ik (p_i beta_k^T) / sum_k w_ik,
 *   w_ik  = exp(-|x_k - x_i|^2 / (2 sigma_s^2)) * exp(-|yhat_k - yhat_i|^2 / (2 sigma_r^2)),
 * where yhat_k = p_k beta_k^T is the temporal output of pixel k (Eq. 6) and
 * |.| is the Euclidean norm (pixels; RGB).  sigma = +inf turns its factor
 * off.  feats: the features of the frame just stepped ((d-1) planes; unused
 * in paper mode).  out: planar [3][H][W].  Returns -1 before the first step
 * or without features.
 */
int oracle_blend(const oracle *o, const double *feats, double sigma_s, double sigma_r, double *out)
{
    int W = o->W, H = o->H, d = o->d;
    size_t n = npix(o);
    if (o->frames == 0) return -1;
    if (o->wmode != ORACLE_W_PAPER && d > 1 && !feats) return -1;
    double *yhat = malloc(n * 3 * sizeof(double));
    if (!yhat) return -1;
    for (size_t j = 0; j < n; j++) {
        double p[32];
        blend_predictor(o, feats, j, p);
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int m = 0; m < d; m++) acc += p[m] * o->beta_cur[j * 3 * d + (size_t)c * d + m];
            yhat[j * 3 + c] = acc;
        }
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            size_t i = (size_t)y * W + x;
            double p[32], num[3] = {0.0, 0.0, 0.0}, den = 0.0;
            blend_predictor(o, feats, i, p);
            for (int dy = -2; dy <= 2; dy++) {
                for (int dx = -2; dx <= 2; dx++) {
                    int nx = x + dx, ny = y + dy;
                    if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
                    size_t k = (size_t)ny * W + nx;
                    double ds2 = (double)(dx * dx + dy * dy);
                    double dr2 = 0.0;
                    for (int c = 0; c < 3; c++) {
                        double e = yhat[k * 3 + c] - yhat[i * 3 + c];
                        dr2 += e * e;
                    }
                    double w = exp(-ds2 / (2.0 * sigma_s * sigma_s)) *
                               exp(-dr2 / (2.0 * sigma_r * sigma_r));
                    for (int c = 0; c < 3; c++) {
                        double pred = 0.0;  /* neighbour k's model at pixel i */
                        for (int m = 0; m < d; m++)
                            pred += p[m] * o->beta_cur[k * 3 * d + (size_t)c * d + m];
                        num[c] += w * pred;
                    }
                    den += w;
                }
            }
            for (int c = 0; c < 3; c++) out[(size_t)c * n + i] = num[c] / den;
        }
    }
    free(yhat);
    return 0;
}
