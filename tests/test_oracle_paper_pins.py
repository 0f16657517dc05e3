"""Pins of the oracle's paper mode (Sec. 5.3): temporal feature (Eq. 12),
feature-based weight (Eq. 13), predictor p = [1, z] with d = 4.

* With the clamp unable to bind (every 3x3 neighbourhood spans the full
  value range), Eq. 12 is an exponential moving average of the colour.
* The clamp Psi limits the reprojected history to the 3x3 neighbourhood
  range of the current colour (checked against a library min/max filter).
* A pixel without history has z = colour, so Eq. 13 gives weight 1.
* With a huge bandwidth h every weight is 1: the model is plain RLS on
  p = [1, z] and matches the closed-form least squares.
* The history is reprojected like the model: bilinear on a bilinear field.
* A non-finite colour carries the history unchanged and only ages P.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle

ALPHA = 0.75


def _checker(T, H, W, lo=0.2, hi=1.0):
    """Colour whose every 3x3 neighbourhood contains both lo and hi."""
    y, x = np.mgrid[0:H, 0:W]
    out = np.empty((T, 3, H, W))
    for t in range(T):
        for c in range(3):
            out[t, c] = np.where((x + y + t + c) % 2 == 0, lo, hi)
    return out


def _closed_form(pseq, yseq, lam, delta=1.0):
    T, d = pseq.shape
    A = lam ** T * delta * np.eye(d)
    b = np.zeros((d, 3))
    for k in range(T):
        A += lam ** (T - 1 - k) * np.outer(pseq[k], pseq[k])
        b += lam ** (T - 1 - k) * np.outer(pseq[k], yseq[k])
    return np.linalg.solve(A, b).T


def test_history_is_ema_and_huge_bandwidth_is_plain_rls():
    T, H, W, lam = 9, 5, 6, 0.95
    col = _checker(T, H, W)
    o = oracle.Oracle(W, H, 4, lam=lam, wmode=oracle.W_PAPER, h_bw=1e9)
    zs = []
    for t in range(T):
        out = o.step(col[t], None, None)
        zs.append(o.get_history())
    ema = col[0].copy()
    for t in range(T):
        if t > 0:
            ema = ALPHA * ema + (1 - ALPHA) * col[t]
        np.testing.assert_allclose(zs[t], ema, rtol=0, atol=1e-15)
    _, beta = o.get_state()
    for y in range(H):
        for x in range(W):
            pseq = np.array([[1.0, *zs[t][:, y, x]] for t in range(T)])
            b = _closed_form(pseq, col[:, :, y, x], lam)
            np.testing.assert_allclose(beta[:, :, y, x], b, rtol=1e-7, atol=1e-9)
            np.testing.assert_allclose(out[:, y, x], b @ pseq[-1], rtol=1e-9, atol=1e-12)


def test_clamp_limits_history_to_neighbourhood_range():
    rng = np.random.default_rng(20)
    H, W = 7, 8
    o = oracle.Oracle(W, H, 4, wmode=oracle.W_PAPER)
    hist = rng.uniform(-3, 3, size=(3, H, W))
    P0 = np.broadcast_to(np.eye(4)[:, :, None, None], (4, 4, H, W))
    o.set_state(P0, np.zeros((3, 4, H, W)), frames=1)
    o.set_history(hist)
    col = rng.uniform(0.0, 1.0, size=(3, H, W))
    o.step(col, None, None)
    z = o.get_history()
    lo = np.stack([ndimage.minimum_filter(col[c], size=3, mode="nearest") for c in range(3)])
    hi = np.stack([ndimage.maximum_filter(col[c], size=3, mode="nearest") for c in range(3)])
    expect = ALPHA * np.clip(hist, lo, hi) + (1 - ALPHA) * col
    np.testing.assert_allclose(z, expect, rtol=0, atol=1e-15)
    assert np.any(hist > hi) and np.any(hist < lo)   # the clamp did bind


def test_no_history_gives_feature_equal_colour_and_unit_weight():
    rng = np.random.default_rng(21)
    H, W, lam = 4, 5, 0.9
    col = rng.uniform(0.1, 2.0, size=(3, H, W))
    o = oracle.Oracle(W, H, 4, lam=lam, wmode=oracle.W_PAPER)
    out, prior = o.step(col, None, None, want_prior=True)
    np.testing.assert_array_equal(o.get_history(), col)
    # w = 1 at P = I: y - yhat = e * lam / (lam + |p|^2)
    p2 = 1.0 + np.sum(col ** 2, axis=0)
    np.testing.assert_allclose(col - out, (col - prior) * lam / (lam + p2), rtol=1e-12)


def test_weight_follows_eq13_on_a_second_frame():
    rng = np.random.default_rng(22)
    H, W, lam, h = 5, 5, 0.97, 0.75
    o = oracle.Oracle(W, H, 4, lam=lam, wmode=oracle.W_PAPER, h_bw=h)
    o.step(rng.uniform(0.2, 1.0, size=(3, H, W)), None, None)
    P_prev, _ = o.get_state()
    col = rng.uniform(0.2, 1.0, size=(3, H, W)) * rng.choice([1.0, 3.0], size=(1, H, W))
    out, prior = o.step(col, None, None, want_prior=True)
    z = o.get_history()
    dist = np.linalg.norm(col - z, axis=0) / (np.minimum(np.linalg.norm(col, axis=0),
                                                         np.linalg.norm(z, axis=0)) + 1e-4)
    w = np.exp(-dist ** 2 / h ** 2)
    p = np.concatenate([np.ones((1, H, W)), z])
    s = np.einsum("ihw,ijhw,jhw->hw", p, P_prev, p)
    np.testing.assert_allclose(col - out, (col - prior) * lam / (lam + w * s), rtol=1e-9, atol=1e-15)
    assert w.min() < 0.9 < w.max()   # weights actually vary


def test_history_reprojects_bilinearly():
    """Unbindable clamp (colour +-100 checkerboard): z = a zq + (1-a) I, so
    zq = (z - (1-a) I)/a must equal the bilinear history field at j + v."""
    rng = np.random.default_rng(23)
    H, W = 8, 9
    o = oracle.Oracle(W, H, 4, wmode=oracle.W_PAPER)
    X = np.arange(W)[None, :]
    Y = np.arange(H)[:, None]
    a, b, c, e = rng.uniform(-1, 1, size=(4, 3, 1, 1))
    hist = a + b * X + c * Y + e * X * Y
    o.set_state(np.broadcast_to(np.eye(4)[:, :, None, None], (4, 4, H, W)),
                np.zeros((3, 4, H, W)), frames=1)
    o.set_history(hist)
    col = 100.0 * (2.0 * (_checker(1, H, W, 0.0, 1.0)[0]) - 1.0)
    tx = rng.uniform(0, W - 1, size=(H, W))
    ty = rng.uniform(0, H - 1, size=(H, W))
    motion = np.stack([tx - X, ty - Y]).astype(np.float32).astype(np.float64)
    o.step(col, None, None, motion)
    zq = (o.get_history() - (1 - ALPHA) * col) / ALPHA
    sx, sy = X + motion[0], Y + motion[1]  # j + v, exact in binary64 here
    np.testing.assert_allclose(zq, a + b * sx + c * sy + e * sx * sy, rtol=1e-10, atol=1e-10)


def test_nonfinite_colour_carries_history_and_ages_model():
    rng = np.random.default_rng(24)
    H, W, lam = 4, 4, 0.8
    o = oracle.Oracle(W, H, 4, lam=lam, wmode=oracle.W_PAPER)
    o.step(rng.uniform(0.2, 1.0, size=(3, H, W)), None, None)
    P1, B1 = o.get_state()
    z1 = o.get_history()
    col = rng.uniform(0.2, 1.0, size=(3, H, W))
    col[1, 2, 3] = np.nan
    o.step(col, None, None)
    P2, B2 = o.get_state()
    np.testing.assert_array_equal(o.get_history()[:, 2, 3], z1[:, 2, 3])
    np.testing.assert_allclose(P2[:, :, 2, 3], P1[:, :, 2, 3] / lam, rtol=1e-15)
    np.testing.assert_array_equal(B2[:, :, 2, 3], B1[:, :, 2, 3])


def test_paper_mode_requires_d4():
    with pytest.raises(ValueError):
        oracle.Oracle(8, 8, 8, wmode=oracle.W_PAPER)
