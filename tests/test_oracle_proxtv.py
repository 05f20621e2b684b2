"""Pins of the oracle's proximal-TV denoiser (Sec. 6, "Proximal-based TV
denoiser"; the map is K fast gradient projection steps on the TV dual).

What fixes it independently of its own code: the adjoint identity of the
discrete gradient; special cases (constant images, lam -> 0, large lam ->
the mean); a one-row image, where isotropic TV is 1D TV and the dual is a
box-constrained least-squares problem solved exactly by scipy's bounded
least squares; and the primal-dual gap of a converged 2D run, which vanishes
only if the gradient, its adjoint and the projection agree.
"""
import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

from oracle import denoisers as den


def test_gradient_adjoint_identity():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((9, 7))
    q1, q2 = rng.standard_normal((9, 7)), rng.standard_normal((9, 7))
    g1, g2 = den.grad_fwd(u)
    lhs = float(np.sum(g1 * q1 + g2 * q2))
    rhs = float(np.sum(u * den.grad_adj(q1, q2)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
    # the last row / column carry no difference
    assert np.all(g1[-1, :] == 0.0) and np.all(g2[:, -1] == 0.0)


def test_tv_of_simple_images():
    x = np.zeros((4, 4))
    x[:, 2:] = 1.0  # one vertical edge of height 4
    assert abs(den.tv_iso(x) - 4.0) < 1e-15
    x = np.zeros((3, 3))
    x[1, 1] = 1.0  # centre pixel: two unit differences into it, (1,1) has |(-1,-1)|
    assert abs(den.tv_iso(x) - (2.0 + math.sqrt(2.0))) < 1e-15


def test_constant_image_is_a_fixed_point():
    b = np.full((12, 10), 0.37)
    x = den.prox_tv(b, tau_r=0.04, alpha=0.5, iters=30)
    assert np.array_equal(x, b)


def test_small_lambda_is_nearly_identity():
    b = np.random.default_rng(1).standard_normal((16, 16))
    lam = 1e-7
    x, _ = den.prox_tv_lam(b, lam, 50)
    # x = b - lam grad^T p with |p| <= 1: each entry moves by at most 4 lam
    assert np.max(np.abs(x - b)) <= 4.0 * lam + 1e-15


def test_large_lambda_gives_the_mean():
    b = np.random.default_rng(2).standard_normal((6, 6))
    x, _ = den.prox_tv_lam(b, 50.0, 4000)
    assert np.max(np.abs(x - b.mean())) < 1e-6


@pytest.mark.parametrize("n,lam", [(12, 0.3), (20, 0.8)])
def test_one_row_matches_exact_bounded_least_squares(n, lam):
    """1D TV denoising: x = b - lam D^T p*, p* = argmin ||lam D^T p - b||
    over -1 <= p <= 1, with D the (n-1) x n forward difference."""
    b = np.random.default_rng(n).standard_normal(n)
    D = np.zeros((n - 1, n))
    for j in range(n - 1):
        D[j, j], D[j, j + 1] = -1.0, 1.0
    res = lsq_linear(lam * D.T, b, bounds=(-1.0, 1.0), method="bvls", tol=1e-14)
    x_exact = b - lam * D.T @ res.x
    x, _ = den.prox_tv_lam(b[None, :], lam, 20000)
    assert np.max(np.abs(x[0] - x_exact)) < 1e-6


def test_primal_dual_gap_vanishes():
    b = np.random.default_rng(3).standard_normal((16, 16))
    lam = 0.3
    x, (p1, p2) = den.prox_tv_lam(b, lam, 3000)
    primal = 0.5 * np.sum((x - b) ** 2) + lam * den.tv_iso(x)
    dual = 0.5 * np.sum(b * b) - 0.5 * np.sum((b - lam * den.grad_adj(p1, p2)) ** 2)
    assert np.max(np.sqrt(p1 * p1 + p2 * p2)) <= 1.0 + 1e-12
    assert 0.0 <= primal - dual <= 1e-9 * primal


def test_planted_adjoint_mistake_is_caught(monkeypatch):
    """A sign slip in the adjoint (a plausible mistake) leaves a visible gap."""
    b = np.random.default_rng(4).standard_normal((12, 12))
    good = den.grad_adj
    monkeypatch.setattr(den, "grad_adj", lambda p1, p2: -good(p1, p2))
    x, (p1, p2) = den.prox_tv_lam(b, 0.3, 500)
    primal = 0.5 * np.sum((x - b) ** 2) + 0.3 * den.tv_iso(x)
    dual = 0.5 * np.sum(b * b) - 0.5 * np.sum((b - 0.3 * good(p1, p2)) ** 2)
    assert abs(primal - dual) > 1e-3 * primal


def test_momentum_sequence():
    beta = den.fgp_momentum(4)
    # t = 1, 1.618..., 2.193..., 2.749..., 3.30...
    t = [1.0]
    for _ in range(4):
        t.append((1.0 + math.sqrt(1.0 + 4.0 * t[-1] ** 2)) / 2.0)
    assert beta[0] == 0.0
    assert all(abs(beta[k] - (t[k] - 1.0) / t[k + 1]) < 1e-15 for k in range(4))
