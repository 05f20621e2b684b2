"""Pins of the oracle's plug-in denoisers and the MC divergence (Sec. 4.3)."""
import math

import numpy as np

from oracle import denoisers as den


def test_haar_orthonormal_and_invertible():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((32, 32))
    for J in (1, 3):
        c = den.haar_fwd(x, J)
        assert abs(np.sum(c * c) - np.sum(x * x)) < 1e-10
        assert np.max(np.abs(den.haar_inv(c, J) - x)) < 1e-12


def test_haar_coefficients_closed_form():
    # a constant image has only its coarse approximation; one level of a 2x2 block is its
    # scaled sum / differences
    c = den.haar_fwd(np.full((8, 8), 2.0), 3)
    assert abs(c[0, 0] - 2.0 * 8) < 1e-12 and np.count_nonzero(np.abs(c) > 1e-12) == 1
    x = np.array([[1.0, 2.0], [3.0, 5.0]])
    c = den.haar_fwd(x, 1)
    assert np.allclose(c, [[11 / 2, -3 / 2], [-5 / 2, 1 / 2]])


def test_haar_soft_divergence_brute_force():
    rng = np.random.default_rng(1)
    I, tau = 16, 0.3
    r = rng.standard_normal((I, I))
    exact = den.haar_soft_exact_div(r, tau, 1.5)
    h = 1e-7
    D0 = den.haar_soft(r, tau, 1.5)
    tr = 0.0
    for k in range(I * I):
        e = np.zeros(I * I)
        e[k] = h
        tr += (den.haar_soft(r + e.reshape(I, I), tau, 1.5).ravel()[k] - D0.ravel()[k]) / h
    assert abs(tr / (I * I) - exact) < 1e-6


def test_mc_divergence_unbiased():
    rng = np.random.default_rng(2)
    I, tau = 32, 0.2
    r = rng.standard_normal((I, I))
    exact = den.haar_soft_exact_div(r, tau, 1.5)
    x = den.haar_soft(r, tau, 1.5)
    est = np.array([den.mc_divergence(den.HAAR, r, tau, dict(alpha=1.5), x, 7, t, 1e-6)[0]
                    for t in range(1000)])
    se = est.std(ddof=1) / math.sqrt(est.size)
    assert abs(est.mean() - exact) < 3 * se + 1e-9


def test_nlm_constant_image_is_fixed_point():
    r = np.full((40, 40), 0.37)
    assert np.max(np.abs(den.nlm(r, 0.01) - r)) < 1e-13


def test_nlm_small_sigma_is_identity():
    rng = np.random.default_rng(3)
    r = rng.standard_normal((32, 32))
    assert np.max(np.abs(den.nlm(r, 1e-8) - r)) < 1e-12


def test_nlm_large_sigma_is_box_filter_with_symmetric_borders():
    # all weights -> 1: the search-window mean, borders extended half-sample symmetrically
    from scipy.ndimage import uniform_filter
    rng = np.random.default_rng(4)
    r = rng.standard_normal((30, 30))
    ref = uniform_filter(r, size=21, mode="reflect")
    assert np.max(np.abs(den.nlm(r, 1e8) - ref)) < 1e-9


def test_nlm_transpose_equivariant():
    rng = np.random.default_rng(5)
    r = rng.standard_normal((36, 36))
    assert np.max(np.abs(den.nlm(r.T, 0.5) - den.nlm(r, 0.5).T)) < 1e-13


# Hand-derived values of the non-local-means weights (the patch-based plug-in's
# reading: d2 = MEAN squared difference over the (2pr+1)^2 patch, weight
# exp(-max(d2 - 2 sigma^2, 0) / (0.4 sigma)^2)).  At pixel (2, 2) of a 5 x 5
# image with pr = sr = 1 neither the patch nor the search window touches the
# border, so no reflection enters.  The numbers below were worked out by hand
# from those definitions; a summed (not averaged) d2, h = 0.4 sigma^2, or a
# dropped 2 sigma^2 offset each changes them by orders of magnitude.

def _step_image(c3, c4):
    r = np.zeros((5, 5))
    r[:, 3] = c3
    r[:, 4] = c4
    return r


def test_nlm_weights_hand_computed_step():
    # columns 3, 4 hold 1: the patch at (2, 2) reads [0 0 1] in each row.  Offsets with
    # dj = -1 ([0 0 0]) and dj = +1 ([0 1 1]) differ in one pixel per row: d2 = 3/9 = 1/3;
    # dj = 0 gives d2 = 0.  Only dj = +1 lands on a 1, so out = w1 / (1 + 2 w1).
    # sigma = 0.4: 2 sigma^2 = 8/25, h^2 = 16/625, (1/3 - 8/25) / (16/625) = 25/48,
    # w1 = e^(-25/48) = 0.59402532055363..., out = 0.27148609332598...
    out = den.nlm(_step_image(1.0, 1.0), 0.4 ** 2, pr=1, sr=1, hfac=0.4)
    assert abs(out[2, 2] - 0.27148609332598) < 1e-12
    # sigma = 0.5: 2 sigma^2 = 1/2 > 1/3, the max(., 0) clamp makes every weight 1, so
    # out is the plain 3 x 3 window mean 3/9.
    out = den.nlm(_step_image(1.0, 1.0), 0.5 ** 2, pr=1, sr=1, hfac=0.4)
    assert abs(out[2, 2] - 1.0 / 3.0) < 1e-14
    # sigma = 0.3: 2 sigma^2 = 9/50, h^2 = 9/625, (1/3 - 9/50) / (9/625) = 575/54,
    # w1 = e^(-575/54) = 2.37447727e-5, out = w1 / (1 + 2 w1)
    out = den.nlm(_step_image(1.0, 1.0), 0.3 ** 2, pr=1, sr=1, hfac=0.4)
    assert abs(out[2, 2] - 2.3743645134642e-05) < 1e-16


def test_nlm_weights_hand_computed_ramp():
    # column 3 = 1, column 4 = 2: dj = -1 gives d2 = 1/3, dj = +1 ([0 1 2] against [0 0 1])
    # gives 6/9 = 2/3, dj = 0 gives 0; only dj = +1 lands on a non-zero pixel (value 1):
    # out = w2 / (1 + w1 + w2).  sigma = 0.5: w0 = w1 = 1 (clamped),
    # w2 = e^(-(2/3 - 1/2) / (1/25)) = e^(-25/6) = 0.015503853599009..., out = 0.0076922966787...
    out = den.nlm(_step_image(1.0, 2.0), 0.5 ** 2, pr=1, sr=1, hfac=0.4)
    assert abs(out[2, 2] - 0.0076922966787311) < 1e-14
