"""GAMP output channel for the Poisson transmission model, FP64 (test infrastructure).

Model (Sec. 2.1 eq. Poisson_CT, Sec. 4.2 eq. noise_mod): Y ~ Poisson(I0 e^-z).
For one ray, GAMP's scalar posterior of z given p, y, tau_p is
    q(z) ~ exp(L(z)),  L(z) = -(z - p)^2 / (2 tau_p) - y z - I0 e^-z
(Sec. 3 eq. nonlin_Lik with the likelihood of eq. noise_mod), and the
channel returns (Sec. 3 eq. MMSEm, Sec. 4.2 eq. MMSEmm, Alg. 1 step 2)
    s = (E[z] - p) / tau_p,
    tau_s = 1/(M tau_p) sum_i (1 - Var[z_i] / tau_p).

Appendix A approximates E[z] and Var[z] by Laplace's method around the
stationary point of L.  Readings adopted where the appendix is garbled:
  * I0 is kept in the likelihood (the appendix drops it, which is only
    consistent with I0 = 1);
  * the 1/M factor in front of log p(y|z) is dropped (the appendix's own
    derivative has none);
  * the stationarity condition is -(z - p)/tau_p - y + I0 e^-z = 0 and the
    curvature is L'' = -1/tau_p - I0 e^-z (the appendix prints z/tau_p);
  * z ranges over the real line (the appendix writes R>=0 but its calculus
    ignores the boundary);
  * the moments use the fully exponential Laplace form of the cumulant
    generating function (Tierney, Kass & Kadane 1989), the same order of
    approximation as the appendix's ratio of two Laplace integrals but valid
    for either sign of z:
        E[z]   ~ z0 + L''' sigma^4 / 2
        Var[z] ~ sigma^2 + L'''' sigma^6 / 2 + L'''^2 sigma^8
    with sigma^2 = -1/L''(z0), L''' = lambda, L'''' = -lambda, lambda = I0 e^-z0,
    and Var clamped to [0, tau_p], the interval the exact variance lies in (the
    corrections scale with tau_p and overshoot it when tau_p is large and the
    ray is photon-starved).

The mode has the closed form z0 = p - tau_p y + W0(tau_p I0 e^(tau_p y - p))
(Lambert W).  Its argument overflows, so W0 is evaluated in the log domain:
w solves w + ln w = xi, xi = ln(tau_p I0) + tau_p y - p, by Newton's method
(Corless et al. 1996) to full FP64 precision.

Variants kept for the pins: 'mode' (E = z0, Var = sigma^2), 'tk_ratio'
(Appendix A's literal ratio of two Laplace integrals for E[z] and E[z^2],
interior rays only), 'quad' (exact moments by adaptive quadrature).

Parity: pinned (stationarity, quadrature, the Gaussian/WLS limit of Sec. 2.2
eq. PWLS, positivity of tau_s).
"""
import math

import numpy as np

LAPLACE = 0
MODE_ONLY = 1


def lambert_w_log(xi):
    """w = W0(exp(xi)) for an array xi, never forming exp(xi) for large xi."""
    xi = np.asarray(xi, dtype=np.float64)
    w = np.where(xi > 1.0, xi - np.log(np.maximum(xi, 1.0)), np.exp(np.minimum(xi, 1.0)))
    for _ in range(100):
        # Newton on f(w) = w + ln w - xi:  w <- w (1 + xi - ln w) / (1 + w)
        w_new = w * (1.0 + xi - np.log(w)) / (1.0 + w)
        done = np.all(np.abs(w_new - w) <= 1e-15 * np.abs(w_new))
        w = w_new
        if done:
            break
    return w


def mode(p, y, tau_p, i0):
    """Stationary point z0 of L (Appendix A, corrected stationarity)."""
    p = np.asarray(p, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xi = math.log(tau_p * i0) + tau_p * y - p
    w = lambert_w_log(xi)
    return p - tau_p * y + w


def moments(p, y, tau_p, i0, kind=LAPLACE):
    """(E[z], Var[z]) per ray."""
    z0 = mode(p, y, tau_p, i0)
    lam = i0 * np.exp(-z0)
    sig2 = 1.0 / (1.0 / tau_p + lam)
    if kind == MODE_ONLY:
        return z0, sig2
    d3 = lam          # L'''(z0)
    d4 = -lam         # L''''(z0)
    mean = z0 + 0.5 * d3 * sig2 ** 2
    var = sig2 + 0.5 * d4 * sig2 ** 3 + d3 ** 2 * sig2 ** 4
    # the expansion's corrections grow with tau_p and can leave the interval the exact
    # variance lies in (0 <= Var <= tau_p: the posterior is log-concave with curvature at
    # least 1/tau_p, Brascamp-Lieb); clamp to it
    return mean, np.clip(var, 0.0, tau_p)


def poisson_out(p, y, tau_p, i0, kind=LAPLACE):
    """Alg. 1 step 2: s = (E[z] - p)/tau_p and tau_s (one FP64 scalar)."""
    p = np.asarray(p, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    M = p.size
    mean, var = moments(p, y, tau_p, i0, kind)
    s = (mean - p) / tau_p
    tau_s = np.sum(1.0 - var / tau_p) / (M * tau_p)
    return s, float(tau_s)


# ----------------------------------------------------------------- pins only

def log_post(z, p, y, tau_p, i0):
    return -(z - p) ** 2 / (2.0 * tau_p) - y * z - i0 * np.exp(-z)


def quad_moments(p, y, tau_p, i0, nonneg=False):
    """Exact posterior mean/variance of one ray by adaptive quadrature."""
    from scipy import integrate
    z0 = float(mode(np.array([p]), np.array([y]), tau_p, i0)[0])
    lam = i0 * math.exp(-z0)
    sig = math.sqrt(1.0 / (1.0 / tau_p + lam))
    L0 = float(log_post(z0, p, y, tau_p, i0))
    lo, hi = z0 - 40 * sig, z0 + 40 * sig
    if nonneg:
        lo = max(lo, 0.0)
    f = lambda z, k: (z - z0) ** k * math.exp(float(log_post(z, p, y, tau_p, i0)) - L0)
    pts = [z0] if lo < z0 < hi else None
    m0 = integrate.quad(f, lo, hi, args=(0,), points=pts, epsabs=0, epsrel=1e-13, limit=400)[0]
    m1 = integrate.quad(f, lo, hi, args=(1,), points=pts, epsabs=0, epsrel=1e-13, limit=400)[0]
    m2 = integrate.quad(f, lo, hi, args=(2,), points=pts, epsabs=0, epsrel=1e-13, limit=400)[0]
    mu1 = m1 / m0
    return z0 + mu1, m2 / m0 - mu1 * mu1


def tk_ratio_moments(p, y, tau_p, i0):
    """Appendix A's literal ratio of Laplace integrals (interior rays, z > 0).

    E[z^k] ~ (sigma_k / sigma) exp(L_k(z_k) - L(z0)) with L_k = k ln z + L,
    z_k the maximiser of L_k and sigma_k^2 = -1/L_k''(z_k)."""
    z0 = float(mode(np.array([p]), np.array([y]), tau_p, i0)[0])
    L = lambda z: float(log_post(z, p, y, tau_p, i0))
    sig = math.sqrt(1.0 / (1.0 / tau_p + i0 * math.exp(-z0)))

    def kth(k):
        z = max(z0, 1e-3)
        for _ in range(200):
            g = k / z - (z - p) / tau_p - y + i0 * math.exp(-z)
            gp = -k / z ** 2 - 1.0 / tau_p - i0 * math.exp(-z)
            step = g / gp
            zn = z - step
            if zn <= 0:
                zn = 0.5 * z
            if abs(zn - z) <= 1e-15 * abs(zn):
                z = zn
                break
            z = zn
        sk = math.sqrt(1.0 / (k / z ** 2 + 1.0 / tau_p + i0 * math.exp(-z)))
        return (sk / sig) * math.exp(k * math.log(z) + L(z) - L(z0))

    e1 = kth(1)
    e2 = kth(2)
    return e1, e2 - e1 * e1
