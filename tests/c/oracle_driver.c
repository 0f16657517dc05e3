/* Drives every entry point of the FP64 oracle (oracle/wrls_oracle.c) over
 * small images with the awkward inputs the tests use -- non-finite colour,
 * features, variance and motion, sources on and past the borders, huge
 * motion, regions of interest, every weight mode, both interpolations, the
 * automatic forgetting factor, state and history export/import -- so that
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer can check
 * its memory accesses and arithmetic.  Exits non-zero on a non-finite
 * output where every input is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle oracle;
oracle *oracle_create(int W, int H, int d, double lambda, double delta, double var_floor,
                      int wmode, int interp);
void oracle_destroy(oracle *o);
void oracle_reset(oracle *o);
long oracle_frames(const oracle *o);
void oracle_set_paper_params(oracle *o, double alpha, double h, double eps);
int oracle_set_forgetting(oracle *o, double sigma0, double lambda_min);
int oracle_threads(void);
void oracle_set_threads(int n);
int oracle_step(oracle *o, const double *color, const double *feats, const double *var,
                const double *motion, double *out, double *prior, double *lam, double *scale,
                int x0, int y0, int x1, int y1);
void oracle_get_state(const oracle *o, double *P, double *beta);
void oracle_get_history(const oracle *o, double *z);
void oracle_set_history(oracle *o, const double *z);
void oracle_get_beta(const oracle *o, double *beta);
void oracle_set_state(oracle *o, const double *P, const double *beta, long frames);
int oracle_blend(const oracle *o, const double *feats, double sigma_s, double sigma_r, double *out);

static unsigned long long rng_state = 12345;
static double uni(void)
{
    rng_state = rng_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

static int run(int W, int H, int d, int wmode, int interp, int autolam)
{
    size_t n = (size_t)W * H;
    int bad = 0;
    oracle *o = oracle_create(W, H, d, 0.95, 1.0, 1e-6, wmode, interp);
    if (!o) return 1;
    if (autolam && oracle_set_forgetting(o, 20.0, 0.4) != 0) bad++;
    double *color = malloc(3 * n * sizeof(double)), *feats = malloc((d > 1 ? d - 1 : 1) * n * sizeof(double));
    double *var = malloc(n * sizeof(double)), *motion = malloc(2 * n * sizeof(double));
    double *out = malloc(3 * n * sizeof(double)), *prior = malloc(3 * n * sizeof(double));
    double *lam = malloc(n * sizeof(double)), *scale = malloc(3 * n * sizeof(double));
    double *P = malloc((size_t)d * d * n * sizeof(double)), *B = malloc(3 * (size_t)d * n * sizeof(double));
    double *z = malloc(3 * n * sizeof(double)), *bl = malloc(3 * n * sizeof(double));
    for (int t = 0; t < 6; t++) {
        int clean = t % 2 == 0;   /* odd frames carry non-finite inputs */
        for (size_t j = 0; j < 3 * n; j++) color[j] = 1.5 * uni();
        for (size_t j = 0; j < (size_t)(d - 1) * n; j++) feats[j] = uni();
        for (size_t j = 0; j < n; j++) var[j] = exp(-3.0 + 2.0 * (uni() - 0.5));
        for (size_t j = 0; j < 2 * n; j++) motion[j] = 3.0 * (uni() - 0.5);
        motion[0] = -1e30;                          /* far outside */
        motion[n - 1] = 0.0;                        /* the last pixel stays in place */
        motion[1 % n] = (double)(W - 1 - (int)(1 % n) % W);   /* exactly onto the last column */
        if (!clean) {
            color[2 % (3 * n)] = NAN;
            color[(n + 3) % (3 * n)] = INFINITY;
            var[4 % n] = -1.0;
            var[5 % n] = INFINITY;
            if (d > 1) feats[6 % n] = NAN;
            motion[n + 7 % n] = NAN;
            motion[8 % n] = -INFINITY;
        }
        int x0 = 0, y0 = 0, x1 = W, y1 = H;
        if (t == 3 && W > 2 && H > 2) { x0 = 1; y0 = 1; x1 = W - 1; y1 = H - 1; }   /* a region of interest */
        if (oracle_step(o, color, d > 1 ? feats : NULL, var, motion, out, prior, lam, scale,
                        x0, y0, x1, y1) != 0) bad++;
        if (clean && t != 3)
            for (size_t j = 0; j < 3 * n; j++)
                if (!isfinite(out[j]) || !isfinite(scale[j])) { bad++; break; }
        for (size_t j = 0; j < n && t != 3; j++)
            if (!(lam[j] > 0.0 && lam[j] <= 1.0)) { bad++; break; }
        if (oracle_blend(o, d > 1 ? feats : NULL, 1.5, t == 4 ? INFINITY : 0.2, bl) != 0) bad++;
    }
    if (oracle_step(o, color, NULL, var, motion, out, NULL, NULL, NULL, 2, 0, 1, H) != -1) bad++;
    oracle_get_state(o, P, B);
    oracle_get_beta(o, B);
    oracle_set_state(o, P, B, 3);
    if (wmode == 2) {
        oracle_get_history(o, z);
        oracle_set_history(o, z);
        oracle_set_paper_params(o, 0.5, 2.0, 1e-3);
    }
    if (oracle_step(o, color, d > 1 ? feats : NULL, var, NULL, out, NULL, NULL, NULL, 0, 0, W, H) != 0) bad++;
    oracle_reset(o);
    if (oracle_frames(o) != 0) bad++;
    if (oracle_blend(o, d > 1 ? feats : NULL, 1.5, 0.2, bl) != -1) bad++;
    oracle_destroy(o);
    free(color); free(feats); free(var); free(motion); free(out); free(prior); free(lam);
    free(scale); free(P); free(B); free(z); free(bl);
    return bad;
}

int main(void)
{
    int bad = 0;
    oracle_set_threads(2);
    if (oracle_threads() != 2) bad++;
    if (oracle_create(0, 4, 2, 0.9, 1.0, 0.0, 0, 0) || oracle_create(4, 4, 8, 0.9, 1.0, 0.0, 2, 0))
        bad++;
    const int dims[][2] = {{13, 7}, {1, 1}, {1, 9}, {9, 1}};
    for (int s = 0; s < 4; s++)
        for (int d = 1; d <= 10; d += (d < 4 ? 3 : (d == 4 ? 4 : 2)))
            for (int wmode = 0; wmode <= 2; wmode++) {
                if (wmode == 2 && d != 4) continue;
                for (int interp = 0; interp <= 1; interp++)
                    for (int autolam = 0; autolam <= 1; autolam++) {
                        int b = run(dims[s][0], dims[s][1], d, wmode, interp, autolam);
                        if (b) printf("case %dx%d d=%d wmode=%d interp=%d auto=%d: %d failures\n",
                                      dims[s][0], dims[s][1], d, wmode, interp, autolam, b);
                        bad += b;
                    }
            }
    printf("oracle driver: %s\n", bad ? "FAILED" : "ok");
    return bad != 0;
}
