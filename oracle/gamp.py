"""GAMP recursion of D-GAMP-CT (Algorithm 1), FP64 (test infrastructure).

Algorithm 1, one iteration t = 0 .. T-1 (the printed "FOR 1..T_max" is read
as T iterations starting from the initial state):
  Step 1  z = Phi~ x^t,  tau_p = ||Phi~||_F^2 tau_x^t / M,  p = z - tau_p s^{t-1}
  Step 2  s^t = (E[z|p,y,tau_p] - p)/tau_p,
          tau_s = 1/(M tau_p) sum (1 - Var[z|p,y,tau_p]/tau_p)
  Step 3  tau_r = N / (||Phi~||_F^2 tau_s),  r = x^t + tau_r Phi~^T s^t
  Step 4  x^{t+1} = D(r),  tau_x^{t+1} = tau_r D'(r)
initialised with x^0 = 0, tau_x^0 = 1 and (unstated in the paper, standard
GAMP) s^{-1} = 0; the result is mu = V^-1 x^T (after the last denoise).
Phi~ = A V^-1 and Phi~^T = V^-1 A^T (Sec. 4.1 eq. precondAMP_op).

Safeguards the paper does not state: a non-positive divergence sets
tau_x = 1e-12 tau_r (counted); a non-finite or non-positive tau stops the
run with an error.  ``onsager=False`` sets p = z (the ablation of Sec. 7).

Damping (Sec. 7 describes x_t = eta_x x^t + (1-eta_x) x^{t-1} and
s^t = eta_r s^t + (1-eta_r) s^{t-1}; the paper ran GAMP through the GAMP
toolbox, whose step size applies the same convex combination to the
variances): from t = 1 on, (s, tau_s) are mixed with their previous values by
eta_s and (x, tau_x) by eta_x.  eta_x = eta_s = 1 is Algorithm 1 verbatim.

The generic ``gamp`` loop is the one both pins and the CT method use: with
an i.i.d. Gaussian Phi, an AWGN output channel and the Bernoulli-Gaussian
MMSE denoiser it must follow the scalar state evolution (Sec. 4.4, Rangan
2011), which fixes the Onsager sign and the ||Phi~||_F^2 / M normalisation.

Parity: the generic loop is pinned by state evolution; the CT instance is
unpinned against the paper (its data are not available) and serves as the
reference for the GPU path.
"""
import math

import numpy as np

from . import channel as _channel
from . import denoisers as _den
from . import precond as _pre
from .probe import rademacher


class GampError(RuntimeError):
    pass


def gamp(forward, adjoint, fro2, M, N, T, out_fn, in_fn, tau_x0=1.0, onsager=True,
         callback=None, eta_x=1.0, eta_s=1.0):
    x = np.zeros(N)
    s = np.zeros(M)
    tau_x = float(tau_x0)
    tau_s = 0.0
    log = []
    clamps = 0
    for t in range(T):
        z = forward(x)
        tau_p = fro2 / M * tau_x
        p = z - tau_p * s if onsager else z
        s_new, tau_s_new = out_fn(p, tau_p)
        if t > 0:
            s = eta_s * s_new + (1.0 - eta_s) * s
            tau_s = eta_s * tau_s_new + (1.0 - eta_s) * tau_s
        else:
            s, tau_s = s_new, tau_s_new
        if not (math.isfinite(tau_s) and tau_s > 0):
            raise GampError("tau_s invalid at iteration %d" % t)
        tau_r = N / (fro2 * tau_s)
        r = x + tau_r * adjoint(s)
        x_new, div = in_fn(r, tau_r, t)
        if div > 0:
            tau_x_new = tau_r * div
        else:
            tau_x_new = 1e-12 * tau_r
            clamps += 1
        if t > 0:
            x = eta_x * x_new + (1.0 - eta_x) * x
            tau_x = eta_x * tau_x_new + (1.0 - eta_x) * tau_x
        else:
            x, tau_x = x_new, tau_x_new
        if not (math.isfinite(tau_x) and tau_x > 0):
            raise GampError("tau_x invalid at iteration %d" % t)
        log.append(dict(t=t, tau_p=tau_p, tau_s=tau_s, tau_r=tau_r, div=div, tau_x=tau_x))
        if callback is not None:
            callback(t, x, log[-1])
    return x, log, clamps


# ------------------------------------------------------------------ D-GAMP-CT

def fro2_exact_dense(A_dense, I):
    """||A V^-1||_F^2 = sum over rays of ||V^-1 a_i||^2 (V^-1 symmetric)."""
    rows = A_dense.reshape(-1, I, I)
    tot = 0.0
    for k in range(0, rows.shape[0], 256):
        f = _pre.apply_Vinv(rows[k:k + 256])
        tot += float(np.sum(f * f))
    return tot


def fro2_hutchinson(radon, n_probes, seed, samples=False):
    """mean over Rademacher probes b_k (probe counter k) of ||A V^-1 b_k||^2
    (E[b b^T] = I makes each term an unbiased estimate of the squared Frobenius norm)."""
    I = radon.I
    vals = []
    for k in range(n_probes):
        b = rademacher(seed, k, I * I).reshape(I, I)
        z = radon.project(_pre.apply_Vinv(b))
        vals.append(float(np.sum(z * z)))
    return vals if samples else float(np.mean(vals))


def dgamp_ct(radon, y, i0, fro2, T, den_kind, den_params, probe_seed, eps_rel=1e-3,
             onsager=True, channel_kind=_channel.LAPLACE, callback=None, eta_x=1.0, eta_s=1.0):
    """Algorithm 1 on the CT model; returns (mu_hat, per-iteration log, clamp count)."""
    I = radon.I
    N, M = I * I, radon.M
    y = np.asarray(y, dtype=np.float64).ravel()

    def forward(x):
        return radon.project(_pre.apply_Vinv(x.reshape(I, I))).ravel()

    def adjoint(s):
        return _pre.apply_Vinv(radon.backproject(s)).ravel()

    def out_fn(p, tau_p):
        return _channel.poisson_out(p, y, tau_p, i0, channel_kind)

    def in_fn(r, tau_r, t):
        r2 = r.reshape(I, I)
        x = _den.apply(den_kind, r2, tau_r, den_params)
        div, _ = _den.mc_divergence(den_kind, r2, tau_r, den_params, x, probe_seed, t, eps_rel)
        return x.ravel(), div

    x, log, clamps = gamp(forward, adjoint, fro2, M, N, T, out_fn, in_fn, onsager=onsager,
                          callback=callback, eta_x=eta_x, eta_s=eta_s)
    return _pre.apply_Vinv(x.reshape(I, I)), log, clamps


# ---------------------------------------------------------- state-evolution pin

def awgn_out(y, sw2):
    """Exact AWGN output channel: s = (y - p)/(tau_p + sw2), tau_s = 1/(tau_p + sw2)."""
    def out_fn(p, tau_p):
        return (y - p) / (tau_p + sw2), 1.0 / (tau_p + sw2)
    return out_fn


def bg_posterior(r, v, rho, sx2):
    """Posterior mean and variance of x ~ (1-rho) delta_0 + rho N(0, sx2) from r = x + N(0, v)."""
    g = sx2 / (sx2 + v)
    ln_on = math.log(rho) - 0.5 * np.log(2 * math.pi * (sx2 + v)) - r * r / (2 * (sx2 + v))
    ln_off = math.log(1 - rho) - 0.5 * np.log(2 * math.pi * v) - r * r / (2 * v)
    pi = 1.0 / (1.0 + np.exp(ln_off - ln_on))
    m = pi * g * r
    var = pi * (g * v + g * g * r * r) - m * m
    return m, var


def bg_denoiser(rho, sx2):
    def in_fn(r, tau_r, t):
        m, var = bg_posterior(r, tau_r, rho, sx2)
        return m, float(np.mean(var)) / tau_r
    return in_fn


def bg_mmse(v, rho, sx2):
    """E[(x - E[x|r])^2] = E_r[Var(x|r)] for r = x + N(0, v), by adaptive quadrature over r
    (r is a two-component Gaussian mixture)."""
    from scipy import integrate

    def dens(r, var):
        return math.exp(-r * r / (2 * var)) / math.sqrt(2 * math.pi * var)

    def f(r):
        _, pv = bg_posterior(np.array([r]), v, rho, sx2)
        return float(pv[0]) * ((1 - rho) * dens(r, v) + rho * dens(r, sx2 + v))

    L = 12.0 * math.sqrt(sx2 + v)
    knots = [k * math.sqrt(v) for k in (-8, -4, -2, 0, 2, 4, 8)]
    return integrate.quad(f, -L, L, points=knots, limit=400, epsabs=0, epsrel=1e-10)[0]


def se_recursion(rho, sx2, sw2, delta_inv, T, E0):
    """E_{t+1} = mmse(sw2 + (N/M) E_t): the scalar state evolution of GAMP."""
    E = [E0]
    for _ in range(T):
        E.append(bg_mmse(sw2 + delta_inv * E[-1], rho, sx2))
    return E
