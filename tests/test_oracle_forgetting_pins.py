"""Pins of the oracle's automatic forgetting factor (the paper names its
selection as future work, Sec. 7.6; the rule is that of Fortescue,
Kershenbaum and Ydstie, Automatica 1981).

* The rule's defining identity: the weighted a-posteriori error information
  of the fit stays at the prescribed Sigma0.  That information is the
  minimum over beta of the exponentially weighted least-squares cost with
  the per-step factors lambda_t,
      J_t(beta) = L_t (Sigma0 + delta |beta|^2) + sum_k L_{k,t} w_k |y_k - p_k beta|^2,
  L_t the product of lambda_0..lambda_t and L_{k,t} that of
  lambda_{k+1}..lambda_t; it is computed here by a library solve, not by
  the oracle's recursion, and must equal Sigma0 after every frame.
* The recursion applies the factors it reports: beta and P after T frames
  equal the minimiser and the inverse normal matrix of that cost, also when
  the limits bind.
* The constant limits: Sigma0 = +inf, or lam_min = lam, reproduce the
  fixed-lambda closed form at lambda in {0.9, 0.98, 0.998, 1}.
"""
import numpy as np
import pytest

import oracle


def _seq(rng, T, H, W, d, jump_at=None):
    ps = rng.uniform(0.0, 1.0, size=(T, d - 1, H, W))
    ys = rng.uniform(0.0, 1.5, size=(T, 3, H, W))
    var = np.exp(-3.0 + rng.standard_normal((T, H, W)))
    if jump_at is not None:
        ys[jump_at:] += 4.0          # an abrupt change of appearance
    return ps, ys, var


def _cost_minimum(p_seq, y_seq, w_seq, lams, delta, sigma0):
    """min over beta of J_t above for one pixel: p_seq (T,d), y_seq (T,3),
    w_seq (T,), lams (T,) the factors of frames 0..T-1.  Returns (V, beta
    (3,d), P = A^-1)."""
    T, d = p_seq.shape
    L = np.prod(lams)
    A = L * delta * np.eye(d)
    b = np.zeros((d, 3))
    for k in range(T):
        g = np.prod(lams[k + 1:]) * w_seq[k]
        A += g * np.outer(p_seq[k], p_seq[k])
        b += g * np.outer(p_seq[k], y_seq[k])
    beta = np.linalg.solve(A, b).T
    V = L * sigma0 + L * delta * np.sum(beta ** 2)
    for k in range(T):
        g = np.prod(lams[k + 1:]) * w_seq[k]
        V += g * np.sum((y_seq[k] - beta @ p_seq[k]) ** 2)
    return V, beta, np.linalg.inv(A)


def _run(o, ps, ys, var):
    lam_seq = []
    for t in range(ys.shape[0]):
        _, lam = o.step(ys[t], ps[t], var[t], None, want_lambda=True)
        lam_seq.append(lam)
    return np.array(lam_seq)


def test_information_stays_at_sigma0():
    """Unlimited (lambda in [1e-9, 1]): after every frame the minimum of the
    weighted cost, by a library solve with the reported factors, is Sigma0."""
    rng = np.random.default_rng(41)
    T, H, W, d, delta, sigma0 = 10, 3, 4, 3, 1.0, 60.0
    ps, ys, var = _seq(rng, T, H, W, d, jump_at=6)
    var[2, 1, 1] = np.inf            # weight 0: no information, lambda = 1
    o = oracle.Oracle(W, H, d, lam=1.0, delta=delta, sigma0=sigma0, lam_min=1e-9)
    w = np.where(np.isfinite(var), 1.0 / np.maximum(var, 1e-6), 0.0)
    lams = []
    for t in range(T):
        _, lam = o.step(ys[t], ps[t], var[t], None, want_lambda=True)
        lams.append(lam)
        for y in range(H):
            for x in range(W):
                p_seq = np.concatenate([np.ones((t + 1, 1)), ps[:t + 1, :, y, x]], axis=1)
                V, _, _ = _cost_minimum(p_seq, ys[:t + 1, :, y, x], w[:t + 1, y, x],
                                        np.array([l[y, x] for l in lams]), delta, sigma0)
                assert abs(V - sigma0) <= 1e-9 * sigma0, (t, y, x, V)
    lams = np.array(lams)
    assert lams[2, 1, 1] == 1.0
    assert lams.min() < 0.5 < 0.95 < lams.max() <= 1.0   # the jump is forgotten fast


@pytest.mark.parametrize("lam_max,lam_min,sigma0", [(0.98, 0.6, 20.0), (1.0, 0.3, 8.0)])
def test_recursion_applies_reported_factors(lam_max, lam_min, sigma0):
    """beta and P after T frames are the minimiser and the inverse normal
    matrix of the cost with the factors the oracle reports, including
    frames where a limit binds (the lower one in both cases, the upper one
    where it is below 1)."""
    rng = np.random.default_rng(42)
    T, H, W, d, delta = 9, 3, 3, 4, 2.0
    ps, ys, var = _seq(rng, T, H, W, d, jump_at=5)
    o = oracle.Oracle(W, H, d, lam=lam_max, delta=delta, sigma0=sigma0, lam_min=lam_min)
    lams = _run(o, ps, ys, var)
    assert np.any(lams == lam_min)
    assert lam_max == 1.0 or np.any(lams == lam_max)
    assert np.all((lams >= lam_min) & (lams <= lam_max))
    P, beta = o.get_state()
    w = 1.0 / np.maximum(var, 1e-6)
    for y in range(H):
        for x in range(W):
            p_seq = np.concatenate([np.ones((T, 1)), ps[:, :, y, x]], axis=1)
            _, b_ref, P_ref = _cost_minimum(p_seq, ys[:, :, y, x], w[:, y, x], lams[:, y, x],
                                            delta, sigma0)
            np.testing.assert_allclose(beta[:, :, y, x], b_ref, rtol=1e-8, atol=1e-10)
            np.testing.assert_allclose(P[:, :, y, x], P_ref, rtol=1e-8, atol=1e-12)


def _fixed_closed_form(p_seq, y_seq, w_seq, lam, delta):
    T, d = p_seq.shape
    A = (lam ** T) * delta * np.eye(d)
    b = np.zeros((d, 3))
    for k in range(T):
        g = (lam ** (T - 1 - k)) * w_seq[k]
        A += g * np.outer(p_seq[k], p_seq[k])
        b += g * np.outer(p_seq[k], y_seq[k])
    return np.linalg.solve(A, b).T, np.linalg.inv(A)


@pytest.mark.parametrize("lam", [0.9, 0.98, 0.998, 1.0])
@pytest.mark.parametrize("limit", ["sigma0_inf", "lam_min_eq_lam"])
def test_constant_limits_reproduce_fixed_lambda(lam, limit):
    rng = np.random.default_rng(43)
    T, H, W, d, delta = 10, 3, 4, 5, 1.0
    ps, ys, var = _seq(rng, T, H, W, d, jump_at=4)
    kw = dict(sigma0=np.inf, lam_min=0.5 * lam) if limit == "sigma0_inf" else dict(sigma0=5.0, lam_min=lam)
    o = oracle.Oracle(W, H, d, lam=lam, delta=delta, **kw)
    lams = _run(o, ps, ys, var)
    np.testing.assert_allclose(lams, lam, rtol=1e-15)
    P, beta = o.get_state()
    w = 1.0 / np.maximum(var, 1e-6)
    for y in range(H):
        for x in range(W):
            p_seq = np.concatenate([np.ones((T, 1)), ps[:, :, y, x]], axis=1)
            b_ref, P_ref = _fixed_closed_form(p_seq, ys[:, :, y, x], w[:, y, x], lam, delta)
            np.testing.assert_allclose(beta[:, :, y, x], b_ref, rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(P[:, :, y, x], P_ref, rtol=1e-9, atol=1e-12)


def test_fixed_mode_unchanged_and_bad_limits_rejected():
    """sigma0 = 0 (the default) is the fixed factor bitwise; limits outside
    (0, lambda] are refused."""
    rng = np.random.default_rng(44)
    ps, ys, var = _seq(rng, 4, 3, 5, 3)
    a = oracle.Oracle(5, 3, 3, lam=0.95)
    b = oracle.Oracle(5, 3, 3, lam=0.95, sigma0=0.0, lam_min=0.2)
    for t in range(4):
        assert np.array_equal(a.step(ys[t], ps[t], var[t]), b.step(ys[t], ps[t], var[t]))
    with pytest.raises(ValueError):
        oracle.Oracle(5, 3, 3, lam=0.95, sigma0=10.0, lam_min=0.99)
    with pytest.raises(ValueError):
        oracle.Oracle(5, 3, 3, lam=0.95, sigma0=-1.0)
