"""Pins of the FP64 oracle to results fixed by the paper and by mathematics,
not by the oracle itself.

* Closed form: RLS with forgetting factor and weights (Sec. 5.2-5.3, Eq. 8-11
  with the weighted gain of Eq. 14) minimises the exponentially weighted
  least-squares cost with the prior I/delta, so after T frames
      A = lambda^T delta I + sum_k lambda^(T-1-k) w_k p_k^T p_k,
      beta^T = A^-1 sum_k lambda^(T-1-k) w_k p_k^T y_k,   P = A^-1.
  Checked with a library solve, at lambda < 1 and lambda = 1 (batch WLS).
* Unit weights reduce to textbook RLS (Eq. 10); d = 1 reduces to an
  exponentially weighted mean, checked in exact rational arithmetic.
* Brute force: the stacked design matrix of Eq. 7 along integer-motion
  reprojection chains, solved by least squares.
* Invariants: P symmetric positive definite at every frame; noise-free
  reproduction identities; bilinear reprojection exact on bilinear state
  fields; nearest reprojection is a pure gather; reset == fresh stream;
  state export/import resumes bitwise; a region of interest reproduces the
  full frame bitwise.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _inputs(rng, T, H, W, d, var_scale=1.0):
    ps = rng.uniform(0.0, 1.0, size=(T, d - 1, H, W))
    ys = rng.uniform(0.0, 1.5, size=(T, 3, H, W))
    var = var_scale * np.exp(-3.0 + rng.standard_normal((T, H, W)))
    return ps, ys, var


def _closed_form(p_seq, y_seq, w_seq, lam, delta):
    """Exponentially weighted LS with prior delta*I; p_seq (T,d), y_seq (T,3)."""
    T, d = p_seq.shape
    A = (lam ** T) * delta * np.eye(d)
    b = np.zeros((d, 3))
    for k in range(T):
        g = (lam ** (T - 1 - k)) * w_seq[k]
        A += g * np.outer(p_seq[k], p_seq[k])
        b += g * np.outer(p_seq[k], y_seq[k])
    return np.linalg.solve(A, b).T, np.linalg.inv(A)


def _weights(var, floor):
    w = np.where(np.isfinite(var) & (var >= 0), 1.0 / np.maximum(var, floor), 0.0)
    return w


@pytest.mark.parametrize("lam,delta", [(0.98, 1.0), (1.0, 1.0), (0.9, 0.1), (0.998, 3.0)])
def test_closed_form_zero_motion(lam, delta):
    rng = np.random.default_rng(1)
    T, H, W, d = 12, 6, 7, 8
    ps, ys, var = _inputs(rng, T, H, W, d)
    var[3, 2, 2] = np.inf      # an outlier frame: weight 0
    var[5, 1, 4] = -1.0        # invalid variance: weight 0
    var[7, 0, 0] = 1e-9        # below the floor: weight 1/floor
    floor = 1e-6
    o = oracle.Oracle(W, H, d, lam=lam, delta=delta, var_floor=floor)
    for t in range(T):
        out = o.step(ys[t], ps[t], var[t])
    P, beta = o.get_state()
    w = _weights(var, floor)
    worst_b = worst_P = worst_o = 0.0
    for y in range(H):
        for x in range(W):
            pseq = np.concatenate([np.ones((T, 1)), ps[:, :, y, x]], axis=1)
            b_cf, P_cf = _closed_form(pseq, ys[:, :, y, x], w[:, y, x], lam, delta)
            worst_b = max(worst_b, np.abs(beta[:, :, y, x] - b_cf).max() / np.abs(b_cf).max())
            worst_P = max(worst_P, np.abs(P[:, :, y, x] - P_cf).max() / np.abs(P_cf).max())
            o_cf = b_cf @ pseq[-1]
            worst_o = max(worst_o, np.abs(out[:, y, x] - o_cf).max() / np.abs(o_cf).max())
    assert worst_o < 1e-10, worst_o
    assert worst_b < 1e-8, worst_b
    assert worst_P < 1e-8, worst_P


def test_unit_weights_are_textbook_rls():
    """Weight mode ONE is RLS of Eq. 10: the unweighted exponentially
    weighted least-squares solution, whatever variance is supplied."""
    rng = np.random.default_rng(2)
    T, H, W, d = 10, 4, 5, 6
    ps, ys, var = _inputs(rng, T, H, W, d)
    o = oracle.Oracle(W, H, d, lam=0.95, delta=0.5, wmode=oracle.W_ONE)
    for t in range(T):
        out = o.step(ys[t], ps[t], var[t] * 100.0)
    _, beta = o.get_state()
    for y in range(H):
        for x in range(W):
            pseq = np.concatenate([np.ones((T, 1)), ps[:, :, y, x]], axis=1)
            b_cf, _ = _closed_form(pseq, ys[:, :, y, x], np.ones(T), 0.95, 0.5)
            np.testing.assert_allclose(beta[:, :, y, x], b_cf, rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(out[:, y, x], b_cf @ pseq[-1], rtol=1e-11)


def test_d1_is_exponentially_weighted_mean_exact_rationals():
    """d = 1 (intercept only): beta(T) = sum lambda^(T-1-k) w_k y_k /
    (lambda^T delta + sum lambda^(T-1-k) w_k) and P(T) = 1/(denominator),
    compared with exact rational arithmetic on dyadic inputs."""
    lam, delta = Fraction(3, 4), Fraction(1, 2)
    ys = [Fraction(5, 8), Fraction(-3, 4), Fraction(7, 2), Fraction(1, 16), Fraction(9, 4)]
    vs = [Fraction(1, 4), Fraction(2), Fraction(1, 8), Fraction(1), Fraction(1, 2)]
    o = oracle.Oracle(1, 1, 1, lam=float(lam), delta=float(delta), var_floor=1e-9)
    for k in range(len(ys)):
        color = np.full((3, 1, 1), float(ys[k]))
        out = o.step(color, None, np.full((1, 1), float(vs[k])))
        T = k + 1
        den = lam ** T * delta + sum(lam ** (T - 1 - i) / vs[i] for i in range(T))
        num = sum(lam ** (T - 1 - i) / vs[i] * ys[i] for i in range(T))
        P, beta = o.get_state()
        assert abs(beta[0, 0, 0, 0] - float(num / den)) <= 1e-15 * max(1.0, abs(float(num / den)))
        assert abs(P[0, 0, 0, 0] - float(1 / den)) <= 1e-15 * float(1 / den)
        assert out[0, 0, 0] == beta[0, 0, 0, 0]


def _chains_brute_force(ps, ys, var, motion, lam, delta, floor):
    """Eq. 7 stacked along each pixel's reprojection chain (integer motion),
    solved by least squares with the prior rows sqrt(lambda^n delta) I."""
    T, dm1, H, W = ps.shape
    d = dm1 + 1
    w = _weights(var, floor)
    res = np.zeros((3, d, H, W))
    for y in range(H):
        for x in range(W):
            chain = [(T - 1, x, y)]
            t, cx, cy = T - 1, x, y
            while t > 0:
                vx, vy = motion[t, 0, cy, cx], motion[t, 1, cy, cx]
                if not (np.isfinite(vx) and np.isfinite(vy)):
                    break
                sx, sy = cx + int(vx), cy + int(vy)
                if not (0 <= sx < W and 0 <= sy < H):
                    break
                t, cx, cy = t - 1, sx, sy
                chain.append((t, cx, cy))
            n = len(chain)
            rows, rhs = [], []
            for (k, kx, ky) in chain:
                g = np.sqrt(lam ** (T - 1 - k) * w[k, ky, kx])
                rows.append(g * np.concatenate([[1.0], ps[k, :, ky, kx]]))
                rhs.append(g * ys[k, :, ky, kx])
            s = np.sqrt(lam ** n * delta)
            X = np.vstack(rows + [s * np.eye(d)])
            Y = np.vstack(rhs + [np.zeros((d, 3))])
            res[:, :, y, x] = np.linalg.lstsq(X, Y, rcond=None)[0].T
    return res


def test_brute_force_integer_motion_chains():
    rng = np.random.default_rng(3)
    T, H, W, d = 5, 4, 4, 5
    ps, ys, var = _inputs(rng, T, H, W, d)
    motion = rng.integers(-1, 2, size=(T, 2, H, W)).astype(np.float64)
    motion[2, :, 1, 2] = np.nan       # a disoccluded pixel
    motion[3, 0, 0, 3] = np.inf       # a non-finite vector
    lam, delta, floor = 0.9, 2.0, 1e-6
    o = oracle.Oracle(W, H, d, lam=lam, delta=delta, var_floor=floor)
    for t in range(T):
        out = o.step(ys[t], ps[t], var[t], motion[t])
    _, beta = o.get_state()
    ref = _chains_brute_force(ps, ys, var, motion, lam, delta, floor)
    np.testing.assert_allclose(beta, ref, rtol=1e-9, atol=1e-11)
    pred = np.einsum("cdhw,dhw->chw", ref, np.concatenate([np.ones((1, H, W)), ps[-1]]))
    np.testing.assert_allclose(out, pred, rtol=1e-10, atol=1e-12)


def test_P_symmetric_positive_definite_with_subpixel_motion():
    rng = np.random.default_rng(4)
    T, H, W, d = 20, 16, 16, 8
    ps, ys, var = _inputs(rng, T, H, W, d)
    o = oracle.Oracle(W, H, d, lam=0.98, delta=1.0)
    for t in range(T):
        motion = rng.uniform(-1.5, 1.5, size=(2, H, W))
        motion[:, rng.random((H, W)) < 0.05] = np.nan
        o.step(ys[t], ps[t], var[t], motion)
        P, _ = o.get_state()
        M = P.transpose(2, 3, 0, 1).reshape(-1, d, d)
        asym = np.abs(M - M.transpose(0, 2, 1)).max(axis=(1, 2)) / np.abs(M).max(axis=(1, 2))
        assert asym.max() < 1e-12, asym.max()
        np.linalg.cholesky(0.5 * (M + M.transpose(0, 2, 1)))  # raises if not SPD
        assert np.all(np.linalg.eigvalsh(0.5 * (M + M.transpose(0, 2, 1)))[:, 0] > 0)


def test_per_step_residual_identity():
    """y - p beta(t) = (y - p beta(t-1)) * lambda / (lambda + w p P(t-1) p^T)
    at every pixel and frame (Eq. 8, 9, 14 combined)."""
    rng = np.random.default_rng(5)
    T, H, W, d = 6, 5, 6, 8
    ps, ys, var = _inputs(rng, T, H, W, d)
    lam, floor = 0.98, 1e-6
    o = oracle.Oracle(W, H, d, lam=lam, delta=1.0, var_floor=floor)
    for t in range(T):
        P_prev, _ = o.get_state()
        out, prior = o.step(ys[t], ps[t], var[t], want_prior=True)
        p = np.concatenate([np.ones((1, H, W)), ps[t]])
        s = np.einsum("ihw,ijhw,jhw->hw", p, P_prev, p)
        w = _weights(var[t], floor)
        lhs = ys[t] - out
        rhs = (ys[t] - prior) * lam / (lam + w * s)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-14)


def test_noise_free_reproduction():
    """Colour exactly linear in the predictor: beta(T) - beta* equals the
    computable prior bias -A^-1 lambda^T delta beta*; huge weights reproduce
    the noise-free colour."""
    rng = np.random.default_rng(6)
    T, H, W, d = 15, 3, 4, 5
    ps = rng.uniform(0, 1, size=(T, d - 1, H, W))
    bstar = rng.uniform(-1, 1, size=(3, d, H, W))
    p_all = np.concatenate([np.ones((T, 1, H, W)), ps], axis=1)
    ys = np.einsum("cdhw,tdhw->tchw", bstar, p_all)
    var = np.exp(-3 + rng.standard_normal((T, H, W)))
    lam, delta = 0.97, 1.0
    o = oracle.Oracle(W, H, d, lam=lam, delta=delta, var_floor=1e-9)
    for t in range(T):
        o.step(ys[t], ps[t], var[t])
    _, beta = o.get_state()
    w = 1.0 / var
    for y in range(H):
        for x in range(W):
            A = lam ** T * delta * np.eye(d)
            for k in range(T):
                A += lam ** (T - 1 - k) * w[k, y, x] * np.outer(p_all[k, :, y, x], p_all[k, :, y, x])
            bias = -np.linalg.solve(A, lam ** T * delta * bstar[:, :, y, x].T).T
            np.testing.assert_allclose(beta[:, :, y, x] - bstar[:, :, y, x], bias,
                                       rtol=1e-6, atol=1e-12)
    o2 = oracle.Oracle(W, H, d, lam=lam, delta=delta, var_floor=1e-15)
    noisy = ys + rng.standard_normal(ys.shape)
    for t in range(3):
        out = o2.step(noisy[t], ps[t], np.full((H, W), 1e-12))
        assert np.abs(out - noisy[t]).max() < 1e-8


def _bilinear_field(rng, n, H, W):
    a, b, c, e = rng.uniform(-1, 1, size=(4, n, 1, 1))
    X = np.arange(W)[None, None, :]
    Y = np.arange(H)[None, :, None]
    coef = (a, b, c, e)
    return a + b * X + c * Y + e * X * Y, coef


def test_bilinear_reprojection_exact_on_bilinear_fields():
    """Every state entry set to a + b x + c y + e x y: after one step with
    weight 0 the reprojected state equals the field at j + v exactly
    (bilinear interpolation reproduces bilinear functions), P is aged by
    1/lambda and beta is unchanged; pixels with no valid source restart."""
    rng = np.random.default_rng(7)
    H, W, d, lam, delta = 9, 11, 4, 0.9, 2.0
    Pf, Pc = _bilinear_field(rng, d * d, H, W)
    Bf, Bc = _bilinear_field(rng, 3 * d, H, W)
    o = oracle.Oracle(W, H, d, lam=lam, delta=delta)
    o.set_state(Pf.reshape(d, d, H, W), Bf.reshape(3, d, H, W), frames=1)
    xs = np.arange(W)[None, :] + 0 * np.arange(H)[:, None]
    ys_ = np.arange(H)[:, None] + 0 * np.arange(W)[None, :]
    tx = rng.uniform(0, W - 1, size=(H, W))
    ty = rng.uniform(0, H - 1, size=(H, W))
    tx[0, 0], ty[0, 0] = W - 1, H - 1               # exactly on the last pixel
    motion = np.stack([tx - xs, ty - ys_]).astype(np.float32).astype(np.float64)
    motion[0, 1, 1] = W                              # leaves the image
    motion[1, 2, 3] = np.nan                         # disoccluded
    motion[0, 3, 4] = W - 0.5 - 4                    # lands between the last column and W
    motion[1, 3, 4] = 0.0
    sx = xs + motion[0]  # exact in binary64 for these sizes
    sy = ys_ + motion[1]
    p = rng.uniform(0, 1, size=(d - 1, H, W))
    out = o.step(np.zeros((3, H, W)), p, np.full((H, W), np.inf), motion)
    P, beta = o.get_state()
    a, b, c, e = Pc
    Pexp = ((a + b * sx + c * sy + e * sx * sy) / lam).reshape(d, d, H, W)
    a, b, c, e = Bc
    Bexp = (a + b * sx + c * sy + e * sx * sy).reshape(3, d, H, W)
    for (yy, xx) in [(1, 1), (2, 3), (3, 4)]:
        Pexp[:, :, yy, xx] = np.eye(d) / delta / lam
        Bexp[:, :, yy, xx] = 0.0
    np.testing.assert_allclose(P, Pexp, rtol=1e-12, atol=1e-11)
    np.testing.assert_allclose(beta, Bexp, rtol=1e-12, atol=1e-11)
    pfull = np.concatenate([np.ones((1, H, W)), p])
    np.testing.assert_allclose(out, np.einsum("cdhw,dhw->chw", Bexp, pfull), rtol=1e-12, atol=1e-11)


def test_nearest_reprojection_is_a_gather():
    rng = np.random.default_rng(8)
    H, W, d, lam = 7, 9, 3, 0.95
    P0 = rng.standard_normal((d, d, H, W))
    B0 = rng.standard_normal((3, d, H, W))
    o = oracle.Oracle(W, H, d, lam=lam, interp=oracle.INTERP_NEAREST)
    o.set_state(P0, B0, frames=3)
    motion = rng.uniform(-2.5, 2.5, size=(2, H, W)).astype(np.float32).astype(np.float64)
    motion[:, 0, 0] = (0.5, 0.5)  # rounds half up
    o.step(np.zeros((3, H, W)), rng.uniform(size=(d - 1, H, W)), np.full((H, W), np.inf), motion)
    P, beta = o.get_state()
    for y in range(H):
        for x in range(W):
            sx = Fraction(x) + Fraction(float(motion[0, y, x]))
            sy = Fraction(y) + Fraction(float(motion[1, y, x]))
            if 0 <= sx <= W - 1 and 0 <= sy <= H - 1:
                xn, yn = int(np.floor(sx + Fraction(1, 2))), int(np.floor(sy + Fraction(1, 2)))
                assert np.array_equal(P[:, :, y, x], P0[:, :, yn, xn] / lam)
                assert np.array_equal(beta[:, :, y, x], B0[:, :, yn, xn])
            else:
                assert np.array_equal(P[:, :, y, x], np.eye(d) / lam)
    P, _ = o.get_state()
    assert np.array_equal(P[:, :, 0, 0], P0[:, :, 1, 1] / lam)


def test_reset_equals_fresh_stream():
    rng = np.random.default_rng(9)
    T, H, W, d = 8, 5, 5, 8
    ps, ys, var = _inputs(rng, T, H, W, d)
    motion = rng.uniform(-1, 1, size=(T, 2, H, W))
    a = oracle.Oracle(W, H, d)
    for t in range(5):
        a.step(ys[t], ps[t], var[t], motion[t])
    a.reset()
    b = oracle.Oracle(W, H, d)
    for t in range(5, T):
        oa = a.step(ys[t], ps[t], var[t], motion[t])
        ob = b.step(ys[t], ps[t], var[t], motion[t])
        assert np.array_equal(oa, ob)
    # a pixel whose motion is NaN restarts exactly like a fresh stream
    m = motion[T - 1].copy()
    m[:, 2, 3] = np.nan
    c = oracle.Oracle(W, H, d)
    fresh = c.step(ys[T - 1], ps[T - 1], var[T - 1])
    out = a.step(ys[T - 1], ps[T - 1], var[T - 1], m)
    assert np.array_equal(out[:, 2, 3], fresh[:, 2, 3])


def test_state_export_import_resumes_bitwise():
    rng = np.random.default_rng(10)
    T, H, W, d = 7, 6, 5, 8
    ps, ys, var = _inputs(rng, T, H, W, d)
    motion = rng.uniform(-1, 1, size=(T, 2, H, W))
    a = oracle.Oracle(W, H, d)
    for t in range(4):
        a.step(ys[t], ps[t], var[t], motion[t])
    P, beta = a.get_state()
    b = oracle.Oracle(W, H, d)
    b.set_state(P, beta, frames=4)
    for t in range(4, T):
        assert np.array_equal(a.step(ys[t], ps[t], var[t], motion[t]),
                              b.step(ys[t], ps[t], var[t], motion[t]))


def test_region_of_interest_matches_full_frame():
    """Stepping only the backward footprint of a window reproduces the full
    computation inside the window bitwise."""
    rng = np.random.default_rng(11)
    T, H, W, d = 6, 20, 24, 8
    ps, ys, var = _inputs(rng, T, H, W, d)
    motion = rng.uniform(-1.7, 1.7, size=(T, 2, H, W))
    full = oracle.Oracle(W, H, d)
    outs = [full.step(ys[t], ps[t], var[t], motion[t]) for t in range(T)]
    win = (10, 8, 14, 12)
    rois = [win]
    for t in range(T - 1, 0, -1):
        x0, y0, x1, y1 = rois[-1]
        m = motion[t, :, y0:y1, x0:x1]
        rois.append((max(0, x0 + int(np.floor(m[0].min()))), max(0, y0 + int(np.floor(m[1].min()))),
                     min(W, x1 + int(np.ceil(m[0].max())) + 1), min(H, y1 + int(np.ceil(m[1].max())) + 1)))
    rois = rois[::-1]
    part = oracle.Oracle(W, H, d)
    for t in range(T):
        o = part.step(ys[t], ps[t], var[t], motion[t], roi=rois[t])
    x0, y0, x1, y1 = win
    assert np.array_equal(o[:, y0:y1, x0:x1], outs[-1][:, y0:y1, x0:x1])


@pytest.mark.parametrize("axis", [0, 1])
def test_crop_reproduces_full_image_bitwise(axis):
    """The source position j + v is evaluated exactly, so it does not depend
    on where the pixel sits: a crop of the image, given the crop's inputs,
    reproduces the full image bitwise for pixels whose motion chains stay
    inside it.  axis 0: a horizontal pan across x ~ 2900; axis 1: a vertical
    pan across y ~ 2900 (where binary32 x + v would be off by up to 1.2e-4)."""
    rng = np.random.default_rng(12)
    T, d, long_, short = 4, 4, 3000, 6
    H, W = (short, long_) if axis == 0 else (long_, short)
    ps, ys, var = _inputs(rng, T, H, W, d)
    motion = np.zeros((T, 2, H, W))
    motion[:, axis] = np.float32(2.3)
    full = oracle.Oracle(W, H, d)
    for t in range(T):
        out_full = full.step(ys[t], ps[t], var[t], motion[t])
    a0, a1 = 2900, 2960
    sl = (slice(None), slice(None), slice(a0, a1)) if axis == 0 else (slice(None), slice(a0, a1), slice(None))
    sl2 = sl[1:]
    cw, ch = (a1 - a0, H) if axis == 0 else (W, a1 - a0)
    crop = oracle.Oracle(cw, ch, d)
    for t in range(T):
        out_crop = crop.step(ys[t][sl], ps[t][sl], var[t][sl2], motion[t][sl])
    n_ok = (a1 - a0) - int(2.3 * T) - 2
    keep = (slice(None), slice(None), slice(0, n_ok)) if axis == 0 else (slice(None), slice(0, n_ok), slice(None))
    assert np.array_equal(out_crop[keep], out_full[sl][keep])


def test_bilinear_reprojection_exact_at_large_coordinates():
    """pi(v_j) = j + v_j holds exactly at the widest accepted image (16384
    pixels), where binary32 spacing is 2^-10 px: every state entry set to a
    bilinear field a + b x + c y + e x y, one weight-0 step with sub-pixel
    motion of either sign, and the reprojected state must equal the field at
    the exact source position; P is aged by 1/lambda.  Sources just past the
    last column by one binary32 ulp of the motion (which a binary32 sum
    x + v would round onto the last column) restart, and a source exactly on
    the last column does not."""
    rng = np.random.default_rng(21)
    H, W, d, lam, delta = 2, 16384, 2, 0.9, 2.0
    Pf, Pc = _bilinear_field(rng, d * d, H, W)
    Bf, Bc = _bilinear_field(rng, 3 * d, H, W)
    o = oracle.Oracle(W, H, d, lam=lam, delta=delta)
    o.set_state(Pf.reshape(d, d, H, W), Bf.reshape(3, d, H, W), frames=1)
    vx = rng.choice(np.array([0.3, -0.7, 1.17, -2.61, 0.013], np.float32), size=(H, W)).astype(np.float64)
    vx[:, :8] = np.abs(vx[:, :8])                       # keep the first columns inside
    vx[:, -8:] = -np.abs(vx[:, -8:])                    # and the last ones
    vy = np.zeros((H, W))
    vy[0] = np.float32(0.25)
    vy[1] = np.float32(-0.75)
    x_edge = W - 3
    up = float(np.nextafter(np.float32(2.0), np.float32(3.0)))  # 2 + 2^-22
    vx[0, x_edge] = 2.0                                   # exactly on the last column
    vx[1, x_edge] = up                                    # 2.4e-7 px past it
    motion = np.stack([vx, vy])
    xs = np.arange(W)[None, :] + np.zeros((H, 1))
    ys_ = np.arange(H)[:, None] + np.zeros((1, W))
    sx, sy = xs + motion[0], ys_ + motion[1]             # exact in binary64 here
    assert float(np.float32(x_edge) + np.float32(up)) == W - 1  # binary32 would call it inside
    p = rng.uniform(0, 1, size=(d - 1, H, W))
    o.step(np.zeros((3, H, W)), p, np.full((H, W), np.inf), motion)
    P, beta = o.get_state()
    a, b, c, e = Pc
    Pexp = ((a + b * sx + c * sy + e * sx * sy) / lam).reshape(d, d, H, W)
    a, b, c, e = Bc
    Bexp = (a + b * sx + c * sy + e * sx * sy).reshape(3, d, H, W)
    Pexp[:, :, 1, x_edge] = np.eye(d) / delta / lam
    Bexp[:, :, 1, x_edge] = 0.0
    np.testing.assert_allclose(P, Pexp, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(beta, Bexp, rtol=1e-12, atol=1e-9)


def test_results_do_not_depend_on_thread_count():
    """Pixels are independent: one thread and many give the same bits."""
    rng = np.random.default_rng(77)
    H, W, d = 9, 23, 4
    frames = [(rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (d - 1, H, W)),
               np.exp(-3 + rng.standard_normal((H, W))), rng.uniform(-1, 1, (2, H, W)))
              for _ in range(4)]
    outs = []
    n0 = oracle.threads()
    try:
        for n in (1, max(2, n0)):
            oracle.set_threads(n)
            o = oracle.Oracle(W, H, d)
            outs.append([o.step(*f) for f in frames] + [o.blend(frames[-1][1], 1.5, 0.2)])
    finally:
        oracle.set_threads(n0)
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)
