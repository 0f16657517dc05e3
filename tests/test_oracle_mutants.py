"""Planted mistakes in the oracle must be caught by its pins.

Each case rewrites one expression of the oracle's C source (a dropped term, a
wrong sign, a swapped index or operand), builds that variant into a temporary
directory, and runs the pin tests against it in a subprocess.  The pins pass
on the real oracle (test_oracle_pins.py) and must fail on every variant.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "wrls_oracle.c")

MUTANTS = {
    "eq14_weight_inverted": ("double den = lambda / w + pPpt;", "double den = lambda * w + pPpt;"),
    "eq14_lambda_dropped": ("double den = lambda / w + pPpt;", "double den = 1.0 / w + pPpt;"),
    "eq8_sign": ("double e = y[c] - pred;", "double e = pred - y[c];"),
    "eq9_sign": ("b[i] += q[i] * e;", "b[i] -= q[i] * e;"),
    "eq11_sign": ("(P[i * d + k] - q[i] * pP[k]) / lambda", "(P[i * d + k] + q[i] * pP[k]) / lambda"),
    "eq11_forgetting": ("(P[i * d + k] - q[i] * pP[k]) / lambda", "(P[i * d + k] - q[i] * pP[k]) * lambda"),
    "weight_is_std": ("return 1.0 / v;", "return 1.0 / sqrt(v);"),
    "prior_inverted": ("(i == k) ? 1.0 / o->delta : 0.0", "(i == k) ? o->delta : 0.0"),
    "reproject_sign": ("source_axis(x, vx, W, nearest, &x0, &fx)", "source_axis(x, -vx, W, nearest, &x0, &fx)"),
    "source_position_binary32": ("    if (!(v >= -(double)j && v <= (double)(n - 1 - j))) return 0;\n",
                                 "    float s32 = (float)j + (float)v;\n"
                                 "    if (!(s32 >= 0.0f && s32 <= (float)(n - 1))) return 0;\n"
                                 "    v = (double)(s32 - (float)j);\n"),
    "bilinear_fraction_sign": ("        *f = v - fl;", "        *f = fl - v + 1.0;"),
    "bilinear_weights_swapped": ("double w10 = fx * (1.0 - fy);\n    double w01 = (1.0 - fx) * fy;",
                                 "double w10 = (1.0 - fx) * fy;\n    double w01 = fx * (1.0 - fy);"),
    "bilinear_tap_transposed": ("size_t s00 = (size_t)y0 * W + x0, s10 = (size_t)y0 * W + x1;",
                                "size_t s00 = (size_t)y0 * W + x0, s10 = (size_t)y1 * W + x0;"),
    "border_check_loose": ("v <= (double)(n - 1 - j)", "v < (double)(n - j)"),
    "nearest_truncates": ("*i0 = j + (int)floor(v + 0.5);", "*i0 = j + (int)floor(v);"),
    "output_a_priori": ("        out[c] = acc;\n", "        out[c] = prior_out ? prior_out[c] : acc;\n"),
    "features_reversed": ("p[i] = feats[(size_t)(i - 1) * n + j];", "p[i] = feats[(size_t)(d - 1 - i) * n + j];"),
    "outlier_not_skipped": ("    if (!isfinite(var) || var < 0.0) return 0.0;\n", ""),
    # automatic forgetting factor (Fortescue, Kershenbaum and Ydstie)
    "vff_root_sign": ("lam = (-B + sqrt(B * B + 4.0 * a)) / 2.0;", "lam = (B + sqrt(B * B + 4.0 * a)) / 2.0;"),
    "vff_error_unweighted": ("double a = w * s, b = w * e2;", "double a = w * s, b = e2;"),
    "vff_gain_term_dropped": ("double B = b / o->sigma0 + a - 1.0;", "double B = b / o->sigma0 - 1.0;"),
    "vff_sigma0_inverted": ("double B = b / o->sigma0 + a - 1.0;", "double B = b * o->sigma0 + a - 1.0;"),
    "vff_upper_limit_ignored": ("    if (lam > o->lambda) lam = o->lambda;\n", ""),
    "vff_lower_limit_ignored": ("    if (lam < o->lambda_min) lam = o->lambda_min;\n", ""),
    "vff_factor_not_applied": ("double lambda = forgetting_factor(o, w, pPpt, y, pred_prior);",
                               "double lambda = o->lambda; (void)forgetting_factor(o, w, pPpt, y, pred_prior);"),
    # paper mode (Eq. 12-13)
    "eq12_alpha_swapped": ("z[c] = o->alpha * psi + (1.0 - o->alpha) * yc[c];",
                           "z[c] = (1.0 - o->alpha) * psi + o->alpha * yc[c];"),
    "eq12_no_clamp": ("double psi = zq[c] < lo ? lo : (zq[c] > hi ? hi : zq[c]);",
                      "double psi = zq[c];"),
    "eq12_clamp_bounds_swapped": ("if (v < lo) lo = v;\n                if (v > hi) hi = v;",
                                  "if (v > lo) lo = v;\n                if (v < hi) hi = v;"),
    "eq12_no_history_is_zero": ("            z[c] = yc[c];\n            continue;",
                                "            z[c] = 0.0;\n            continue;"),
    "eq13_not_squared": ("return exp(-(dist * dist) / (o->h * o->h));", "return exp(-dist / (o->h * o->h));"),
    "eq13_max_norm": ("fmin(sqrt(ny), sqrt(nz))", "fmax(sqrt(ny), sqrt(nz))"),
    "history_reprojection_nearest": ("              + fx * (1.0 - fy) * o->z_prev[((size_t)y0 * W + x1) * 3 + c]",
                                     "              + fx * (1.0 - fy) * o->z_prev[((size_t)y0 * W + x0) * 3 + c]"),
    "history_not_carried": ("                    for (int c = 0; c < 3; c++) z[c] = zq[c];",
                            "                    for (int c = 0; c < 3; c++) z[c] = 0.0;"),
    # spatial blend (Sec. 5.3, last paragraph)
    "blend_window_3x3": ("for (int dy = -2; dy <= 2; dy++) {\n                for (int dx = -2; dx <= 2; dx++) {",
                         "for (int dy = -1; dy <= 1; dy++) {\n                for (int dx = -1; dx <= 1; dx++) {"),
    "blend_spatial_no_half": ("exp(-ds2 / (2.0 * sigma_s * sigma_s))", "exp(-ds2 / (sigma_s * sigma_s))"),
    "blend_range_no_half": ("exp(-dr2 / (2.0 * sigma_r * sigma_r))", "exp(-dr2 / (sigma_r * sigma_r))"),
    "blend_range_dropped": ("exp(-dr2 / (2.0 * sigma_r * sigma_r))", "1.0"),
    "blend_range_l1": ("                        dr2 += e * e;", "                        dr2 += fabs(e);"),
    "blend_neighbour_predictor": ("                            pred += p[m] * o->beta_cur[k * 3 * d + (size_t)c * d + m];",
                                  "                            pred = yhat[k * 3 + c];"),
    "blend_border_clamped": ("                    if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;\n                    size_t k",
                             "                    nx = nx < 0 ? 0 : (nx >= W ? W - 1 : nx);\n"
                             "                    ny = ny < 0 ? 0 : (ny >= H ? H - 1 : ny);\n                    size_t k"),
    "blend_centre_excluded": ("                    size_t k = (size_t)ny * W + nx;\n                    double ds2",
                              "                    if (dx == 0 && dy == 0) continue;\n"
                              "                    size_t k = (size_t)ny * W + nx;\n                    double ds2"),
    "blend_nonfinite_feature_kept": ("p[i] = isfinite(v) ? v : 0.0;", "p[i] = v;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    # a site repeated in the history reprojection is mutated everywhere
    assert src.count(old) >= 1, "mutation site not found: %s" % name
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-w", "-o", str(lib), str(mutant), "-lm"], check=True)
    env = dict(os.environ, WRLS_ORACLE_LIB_OVERRIDE=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_paper_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_forgetting_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_blend_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "planted mistake %r passed every pin:\n%s" % (name, r.stdout[-2000:])
