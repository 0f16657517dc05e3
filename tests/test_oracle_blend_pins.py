"""Pins of the oracle's spatial blend (Sec. 5.3, last paragraph): the final
colour of a pixel i is a bilateral-weighted average, over the 5x5 window
centred on i, of the predictions p_i beta_k^T that the neighbours' models
make for pixel i.

* A spatially constant model makes every prediction equal: the blend returns
  p_i beta^T whatever the weights (the predictor is the centre's, not the
  neighbour's).
* A vanishing spatial width keeps only the centre: the blend returns the
  step's own output.
* With the range factor off, the blend is a normalised 5x5 Gaussian
  filtering of beta (library correlation, zero outside the image, divided by
  the correlation of ones), taken at the centre's predictor; with both
  factors off it is a 5x5 box mean (library uniform filter).
* A two-valued guide whose jump makes the range factor exactly 1/2 gives
  the same filtering with the other region's spatial weights halved (pins
  the Gaussian form, the 2 sigma^2 convention and the squared RGB distance).
* A range width far below an outlier model's jump isolates it; scaling every
  model and the range width by c scales the blend by c (the range factor
  sees colour distance over width).
* Paper mode predicts with p = [1, z] from the stored history.
* Non-finite features enter as 0, as in the step's output.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle


def _gauss5(sigma):
    a = np.arange(-2, 3, dtype=np.float64)
    return np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sigma * sigma))


def _with_state(beta, d, wmode=oracle.W_INVVAR, z=None):
    _, _, H, W = beta.shape
    o = oracle.Oracle(W, H, d, wmode=wmode)
    P = np.broadcast_to(np.eye(d)[:, :, None, None], (d, d, H, W))
    o.set_state(P, beta, frames=1)
    if z is not None:
        o.set_history(z)
    return o


def _pred(p, beta):
    """p (d,H,W), beta (3,d,H,W) -> (3,H,W)."""
    return np.einsum("dhw,cdhw->chw", p, beta)


def _filtered_beta(beta, kernel):
    """Normalised correlation of every beta plane with a 5x5 kernel, zero
    outside the image (the window is cut at the border)."""
    H, W = beta.shape[2:]
    norm = ndimage.correlate(np.ones((H, W)), kernel, mode="constant", cval=0.0)
    out = np.empty_like(beta)
    for c in range(3):
        for m in range(beta.shape[1]):
            out[c, m] = ndimage.correlate(beta[c, m], kernel, mode="constant", cval=0.0) / norm
    return out


def test_constant_model_returns_centre_prediction():
    rng = np.random.default_rng(1)
    H, W, d = 9, 13, 5
    b = rng.uniform(-1, 1, size=(3, d))
    beta = np.broadcast_to(b[:, :, None, None], (3, d, H, W)).copy()
    feats = rng.uniform(-2, 2, size=(d - 1, H, W))
    o = _with_state(beta, d)
    out = o.blend(feats, sigma_s=1.3, sigma_r=0.05)
    p = np.concatenate([np.ones((1, H, W)), feats])
    np.testing.assert_allclose(out, _pred(p, beta), rtol=1e-13, atol=1e-13)


def test_tiny_spatial_width_returns_step_output():
    rng = np.random.default_rng(2)
    H, W, d = 8, 11, 4
    o = oracle.Oracle(W, H, d)
    for _ in range(3):
        feats = rng.uniform(0, 1, size=(d - 1, H, W))
        y = o.step(rng.uniform(0, 1, size=(3, H, W)), feats, np.full((H, W), 0.05),
                   rng.uniform(-0.7, 0.7, size=(2, H, W)))
    out = o.blend(feats, sigma_s=1e-3, sigma_r=np.inf)
    np.testing.assert_array_equal(out, y)


@pytest.mark.parametrize("sigma_s", [0.8, 1.5, 3.0])
def test_range_off_is_normalised_gaussian_filter(sigma_s):
    rng = np.random.default_rng(3)
    H, W, d = 10, 12, 3
    beta = rng.uniform(-1, 1, size=(3, d, H, W))
    feats = rng.uniform(0, 1, size=(d - 1, H, W))
    o = _with_state(beta, d)
    out = o.blend(feats, sigma_s=sigma_s, sigma_r=np.inf)
    p = np.concatenate([np.ones((1, H, W)), feats])
    expect = _pred(p, _filtered_beta(beta, _gauss5(sigma_s)))
    np.testing.assert_allclose(out, expect, rtol=1e-12, atol=1e-12)


def test_both_off_is_box_mean():
    rng = np.random.default_rng(4)
    H, W, d = 7, 9, 2
    beta = rng.uniform(-1, 1, size=(3, d, H, W))
    feats = rng.uniform(0, 1, size=(d - 1, H, W))
    o = _with_state(beta, d)
    out = o.blend(feats, sigma_s=np.inf, sigma_r=np.inf)
    H_, W_ = beta.shape[2:]
    cnt = ndimage.uniform_filter(np.ones((H_, W_)), size=5, mode="constant", cval=0.0)
    box = np.stack([np.stack([ndimage.uniform_filter(beta[c, m], size=5, mode="constant", cval=0.0) / cnt
                              for m in range(d)]) for c in range(3)])
    p = np.concatenate([np.ones((1, H, W)), feats])
    np.testing.assert_allclose(out, _pred(p, box), rtol=1e-12, atol=1e-12)


def test_range_factor_one_half_on_two_valued_guide():
    """Two regions (x < 6 and x >= 6) with constant models A and B, and a
    constant predictor, so the guide (the temporal output) takes two values
    whose RGB distance D is set so that exp(-D^2 / (2 sigma_r^2)) = 1/2."""
    H, W, d = 8, 12, 3
    p0 = np.array([1.0, 0.4, -0.7])
    bA = np.array([[0.2, 0.1, 0.3], [0.5, -0.2, 0.1], [0.0, 0.3, 0.2]])
    bB = bA + np.array([[0.3, 0.0, 0.0], [0.0, 0.25, 0.0], [-0.1, 0.0, 0.2]])
    mA = (np.arange(W)[None, :] < 6) * np.ones((H, 1))
    mB = 1.0 - mA
    beta = bA[:, :, None, None] * mA + bB[:, :, None, None] * mB
    feats = np.broadcast_to(p0[1:, None, None], (d - 1, H, W)).copy()
    D2 = float(np.sum((bA @ p0 - bB @ p0) ** 2))
    sigma_r = np.sqrt(D2 / (2.0 * np.log(2.0)))
    sigma_s = 1.7
    o = _with_state(beta, d)
    out = o.blend(feats, sigma_s=sigma_s, sigma_r=sigma_r)
    G = _gauss5(sigma_s)
    cA = ndimage.correlate(mA, G, mode="constant", cval=0.0)
    cB = ndimage.correlate(mB, G, mode="constant", cval=0.0)
    yA, yB = bA @ p0, bB @ p0
    # a pixel of region A sees region B at half weight, and vice versa
    expect_A = (cA[None] * yA[:, None, None] + 0.5 * cB[None] * yB[:, None, None]) / (cA + 0.5 * cB)[None]
    expect_B = (cB[None] * yB[:, None, None] + 0.5 * cA[None] * yA[:, None, None]) / (cB + 0.5 * cA)[None]
    expect = np.where(mA[None] > 0, expect_A, expect_B)
    np.testing.assert_allclose(out, expect, rtol=1e-12, atol=1e-12)
    # the blend did mix across the edge
    assert np.max(np.abs(out - np.where(mA[None] > 0, yA[:, None, None], yB[:, None, None]))) > 1e-2


def test_paper_mode_predicts_with_history():
    rng = np.random.default_rng(6)
    H, W = 6, 10
    b = rng.uniform(-1, 1, size=(3, 4))
    beta = np.broadcast_to(b[:, :, None, None], (3, 4, H, W)).copy()
    z = rng.uniform(0, 2, size=(3, H, W))
    o = _with_state(beta, 4, wmode=oracle.W_PAPER, z=z)
    out = o.blend(None, sigma_s=2.0, sigma_r=0.3)
    p = np.concatenate([np.ones((1, H, W)), z])
    np.testing.assert_allclose(out, _pred(p, beta), rtol=1e-13, atol=1e-13)


def test_nonfinite_feature_enters_as_zero():
    rng = np.random.default_rng(7)
    H, W, d = 6, 7, 3
    b = rng.uniform(-1, 1, size=(3, d))
    beta = np.broadcast_to(b[:, :, None, None], (3, d, H, W)).copy()
    feats = rng.uniform(0, 1, size=(d - 1, H, W))
    feats[1, 2, 3] = np.nan
    feats[0, 4, 4] = np.inf
    o = _with_state(beta, d)
    out = o.blend(feats, sigma_s=1.0, sigma_r=0.5)
    p = np.concatenate([np.ones((1, H, W)), np.where(np.isfinite(feats), feats, 0.0)])
    assert np.all(np.isfinite(out))
    np.testing.assert_allclose(out, _pred(p, beta), rtol=1e-13, atol=1e-13)


def test_blend_needs_a_state_and_features():
    o = oracle.Oracle(4, 4, 3)
    with pytest.raises(ValueError):
        o.blend(np.zeros((2, 4, 4)), 1.0, 1.0)
    o.step(np.zeros((3, 4, 4)), np.zeros((2, 4, 4)), np.ones((4, 4)))
    with pytest.raises(ValueError):
        o.blend(None, 1.0, 1.0)


def test_small_range_width_rejects_an_outlier_model():
    """One pixel's model differs strongly from its constant surroundings: with
    a range width far below that difference the outlier neither bleeds into
    its neighbours nor takes anything from them."""
    rng = np.random.default_rng(8)
    H, W, d = 9, 9, 3
    b0 = rng.uniform(-0.5, 0.5, size=(3, d))
    beta = np.broadcast_to(b0[:, :, None, None], (3, d, H, W)).copy()
    beta[:, :, 4, 4] += 5.0
    feats = rng.uniform(0.5, 1.0, size=(d - 1, H, W))
    o = _with_state(beta, d)
    out = o.blend(feats, sigma_s=2.0, sigma_r=0.01)
    p = np.concatenate([np.ones((1, H, W)), feats])
    np.testing.assert_allclose(out, _pred(p, beta), rtol=1e-13, atol=1e-13)
    # the same scene with the range factor off does mix
    mixed = o.blend(feats, sigma_s=2.0, sigma_r=np.inf)
    assert np.max(np.abs(mixed - _pred(p, beta))) > 0.1


def test_range_term_depends_on_colour_over_width():
    """Scaling every model (hence every prediction and every colour
    difference) by c and the range width by c scales the blend by c."""
    rng = np.random.default_rng(9)
    H, W, d = 8, 10, 4
    beta = rng.uniform(-1, 1, size=(3, d, H, W))
    feats = rng.uniform(0, 1, size=(d - 1, H, W))
    a = _with_state(beta, d).blend(feats, sigma_s=1.2, sigma_r=0.4)
    c = 7.5
    b = _with_state(c * beta, d).blend(feats, sigma_s=1.2, sigma_r=0.4 * c)
    np.testing.assert_allclose(b, c * a, rtol=1e-12, atol=1e-12)
    # and the range factor is active at this width
    off = _with_state(beta, d).blend(feats, sigma_s=1.2, sigma_r=np.inf)
    assert np.max(np.abs(off - a)) > 1e-2
