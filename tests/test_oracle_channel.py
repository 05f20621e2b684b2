"""Pins of the oracle's Poisson output channel (Sec. 4.2, Appendix A, Alg. 1 step 2)."""
import math

import numpy as np
import pytest

from oracle import channel


def test_lambert_w_matches_library():
    from scipy.special import lambertw
    xi = np.linspace(-30, 40, 301)
    w = channel.lambert_w_log(xi)
    ref = np.real(lambertw(np.exp(xi)))
    assert np.max(np.abs(w - ref) / ref) < 1e-14
    big = np.array([1e3, 1e6, 1e9])
    w = channel.lambert_w_log(big)
    assert np.max(np.abs(w + np.log(w) - big) / big) < 1e-15


def grid():
    out = []
    for i0 in (1e3, 1e4, 1e5):
        for tau_p in (1e-3, 0.1, 10.0, 300.0):
            for zt in (0.0, 0.5, 3.0, 6.0):
                for dp in (-1.0, 0.0, 0.7):
                    y = round(i0 * math.exp(-zt))
                    out.append((zt + dp, float(y), tau_p, i0))
    return out


def test_mode_is_stationary():
    for p, y, tau_p, i0 in grid():
        z0 = float(channel.mode(np.array([p]), np.array([y]), tau_p, i0)[0])
        lam = i0 * math.exp(-z0)
        res = -(z0 - p) / tau_p - y + lam
        # the closed form z0 = p - tau_p y + W(.) cancels terms of size tau_p y, so the implied
        # error of z0 (residual / curvature) is bounded relative to that size
        z_err = abs(res) / (1.0 / tau_p + lam)
        assert z_err <= 1e-14 * (1.0 + tau_p * y + abs(p)), (p, y, tau_p, i0, res)


def test_laplace_moments_vs_quadrature_high_counts():
    worst_m, worst_v = 0.0, 0.0
    for p, y, tau_p, i0 in grid():
        if y < 80:
            continue
        m, v = channel.moments(np.array([p]), np.array([y]), tau_p, i0)
        mq, vq = channel.quad_moments(p, y, tau_p, i0)
        worst_m = max(worst_m, abs(m[0] - mq))
        worst_v = max(worst_v, abs(v[0] - vq) / vq)
    assert worst_m < 3e-6 and worst_v < 3e-5, (worst_m, worst_v)


def test_laplace_beats_mode_only():
    p, y, tau_p, i0 = 0.3, 700.0, 1.0, 1e3
    m, _ = channel.moments(np.array([p]), np.array([y]), tau_p, i0)
    m0, _ = channel.moments(np.array([p]), np.array([y]), tau_p, i0, channel.MODE_ONLY)
    mq, _ = channel.quad_moments(p, y, tau_p, i0)
    assert abs(m[0] - mq) < 0.05 * abs(m0[0] - mq)


def test_tk_ratio_agrees_for_interior_rays():
    for p, y, tau_p, i0 in [(2.0, 1353.0, 0.5, 1e4), (3.1, 450.0, 2.0, 1e4), (1.0, 3.7e4, 0.05, 1e5)]:
        m, v = channel.moments(np.array([p]), np.array([y]), tau_p, i0)
        mt, vt = channel.tk_ratio_moments(p, y, tau_p, i0)
        assert abs(m[0] - mt) < 1e-6 * abs(m[0])
        assert abs(v[0] - vt) < 1e-3 * v[0]


def test_gaussian_wls_limit():
    # Sec. 2.2 eq. PWLS: for large I0 the likelihood is Gaussian in z around ln(I0/y)
    # with precision y; the posterior becomes N(mean, var) of the product of Gaussians.
    for i0 in (1e8, 1e10):
        zt, p, tau_p = 1.3, 1.0, 0.02
        y = float(round(i0 * math.exp(-zt)))
        l = math.log(i0 / y)
        prec = 1.0 / tau_p + y
        mean_ref = (p / tau_p + y * l) / prec
        m, v = channel.moments(np.array([p]), np.array([y]), tau_p, i0)
        assert abs(m[0] - mean_ref) < 1e-7
        assert abs(v[0] * prec - 1.0) < 1e-6


def test_tau_s_positive_and_variance_bounded():
    rng = np.random.default_rng(1)
    for _ in range(20):
        i0 = 10 ** rng.uniform(3, 6)
        tau_p = 10 ** rng.uniform(-4, 3)
        zt = rng.uniform(0, 8, 500)
        y = rng.poisson(i0 * np.exp(-zt)).astype(float)
        p = zt + rng.normal(0, math.sqrt(tau_p), 500)
        _, v = channel.moments(p, y, tau_p, i0)
        assert np.all(v >= 0) and np.all(v <= tau_p)
        s, tau_s = channel.poisson_out(p, y, tau_p, i0)
        assert tau_s > 0 and np.all(np.isfinite(s))


def test_starved_rays_reported_error():
    # y = 0: the Laplace form is the method's approximation; its error is bounded but not tiny.
    for tau_p in (1.0, 10.0):
        m, v = channel.moments(np.array([0.5]), np.array([0.0]), tau_p, 1e4)
        mq, vq = channel.quad_moments(0.5, 0.0, tau_p, 1e4)
        assert abs(m[0] - mq) < 1.0 and 0 < v[0] < tau_p
