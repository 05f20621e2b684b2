"""Pins of the oracle's proximal TV in the (V^T V)^-1 metric (Sec. 4.3 and
Sec. 6 name it for input in the preconditioned domain; the map is K
Chambolle-Pock primal-dual steps, Chambolle & Pock 2011).

What fixes it independently of its own code: with W = I it must reach the
l2 proximal map, which the fast-gradient-projection oracle (another
algorithm, pinned on its own) computes; constant images are fixed points; a
one-row image with a non-trivial circulant W has a dual that is a box-
constrained least-squares problem, solved exactly by scipy's bounded least
squares; and the primal-dual gap of a converged 2D run in the cone metric
vanishes only if the gradient, its adjoint, the metric and the Fourier
division agree.
"""
import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

from oracle import denoisers as den
from oracle import precond


def test_metric_symbol_is_the_inverse_cone_symbol():
    I = 8
    w = den.metric_symbol(I)
    assert abs(w[0, 0] - 1.0 / (4.0 * math.log(1.0 + math.sqrt(2.0)) * I)) < 1e-15
    assert abs(w[0, 1] - 1.0 / I) < 1e-15 and abs(w[3, 4] - 5.0 / I) < 1e-15
    assert np.all(w > 0.0)
    # the figure's reading V^T V: the cone symbol itself
    assert np.array_equal(den.metric_symbol(I, 1), precond.symbol(I))


def test_identity_metric_reaches_the_l2_prox():
    b = np.random.default_rng(0).standard_normal((16, 16))
    x_cp, _ = den.prox_tv_metric(b, 0.3, np.ones((16, 16)), 3000)
    x_fgp, _ = den.prox_tv_lam(b, 0.3, 3000)
    assert np.max(np.abs(x_cp - x_fgp)) < 1e-9


def test_constant_image_is_a_fixed_point():
    b = np.full((12, 12), -0.21)
    x = den.prox_tv_w(b, tau_r=0.05, alpha=1.0, iters=20)
    assert np.max(np.abs(x - b)) < 1e-14


def test_zero_lambda_is_identity():
    b = np.random.default_rng(5).standard_normal((8, 8))
    assert np.array_equal(den.prox_tv_w(b, tau_r=0.0), b)


@pytest.mark.parametrize("n,lam", [(12, 0.3), (16, 0.7)])
def test_one_row_matches_exact_bounded_least_squares(n, lam):
    """min 1/2 (x-b)^T W (x-b) + lam sum |D x| on one row: x = b - lam W^-1 D^T p*,
    p* = argmin over -1 <= p <= 1 of 1/2 ||lam W^-1/2 D^T p - W^1/2 b||^2,
    W the circulant with symbol w (positive, symmetric in k)."""
    rng = np.random.default_rng(n)
    b = rng.standard_normal(n)
    k = np.fft.fftfreq(n) * n
    w = 0.2 + np.abs(k) / n
    F = np.fft.fft(np.eye(n), axis=0)
    Finv = np.conj(F) / n

    def circ(sym):
        return np.real(Finv @ np.diag(sym) @ F)

    D = np.zeros((n - 1, n))
    for j in range(n - 1):
        D[j, j], D[j, j + 1] = -1.0, 1.0
    A = lam * circ(w ** -0.5) @ D.T
    res = lsq_linear(A, circ(w ** 0.5) @ b, bounds=(-1.0, 1.0), method="bvls", tol=1e-14)
    x_exact = b - lam * circ(1.0 / w) @ D.T @ res.x
    x, _ = den.prox_tv_metric(b[None, :], lam, w[None, :], 20000)
    assert np.max(np.abs(x[0] - x_exact)) < 1e-6
    # and the metric matters: the l2 prox of the same row is elsewhere
    x_l2, _ = den.prox_tv_lam(b[None, :], lam, 20000)
    assert np.max(np.abs(x_l2[0] - x_exact)) > 1e-3


def test_primal_dual_gap_vanishes_in_the_cone_metric():
    I = 16
    b = np.random.default_rng(3).standard_normal((I, I))
    lam = 0.3
    w = den.metric_symbol(I)
    x, (p1, p2) = den.prox_tv_metric(b, lam, w, 20000)

    def wnorm2(v, sym):  # v^T F^-1 diag(sym) F v (Parseval with numpy's unnormalised FFT)
        return float(np.sum(sym * np.abs(np.fft.fft2(v)) ** 2) / v.size)

    primal = 0.5 * wnorm2(x - b, w) + lam * den.tv_iso(x)
    a = den.grad_adj(p1, p2)
    dual = lam * float(np.sum(b * a)) - 0.5 * lam * lam * wnorm2(a, 1.0 / w)
    assert np.max(np.sqrt(p1 * p1 + p2 * p2)) <= 1.0 + 1e-12
    assert -1e-9 * abs(primal) <= primal - dual <= 2e-7 * abs(primal)
    # the primal point is the dual's x(p): x = b - lam W^-1 grad^T p
    xp = b - lam * np.real(np.fft.ifft2(np.fft.fft2(a) / w))
    assert np.max(np.abs(xp - x)) < 1e-6 * np.max(np.abs(b))


def test_metric_variant_differs_from_l2_in_the_cone_metric():
    b = np.random.default_rng(7).standard_normal((16, 16)) * 0.1
    x_w = den.prox_tv_w(b, tau_r=0.01, alpha=1.0, iters=200)
    x_2 = den.prox_tv(b, tau_r=0.01, alpha=1.0, iters=200)
    assert np.max(np.abs(x_w - x_2)) > 1e-3
    # the cone metric barely weighs the mean, so TV pulls harder on low frequencies
    assert den.tv_iso(x_w) < den.tv_iso(x_2)
