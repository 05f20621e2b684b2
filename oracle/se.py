"""Scalar state evolution of D-GAMP-CT, FP64 (test infrastructure).

Sec. 4.4 (eqs. SEasym, SE_matches, and the error and sensitivity functions
E_in, A_in): in the large-system limit GAMP's vectors behave like scalar
random variables, and the recursion over the scalars predicts the MSE of
every iterate.  The input side: the denoiser sees R = X + V, V ~ N(0, xi_r);
its error function E_in = (1/N) ||D(x + v) - x||^2 is the predicted MSE of
the next iterate, its sensitivity function A_in (the mean divergence) gives
tau_x = tau_r A_in.  The output side: (Z, P) jointly Gaussian with Z given P
of variance tau_p; in the matched case (the channel is the true likelihood)
xi_r = tau_r = -1 / E[d g_out / dp] (eq. SE_matches).

Readings (the paper states the recursion for an i.i.d. Gaussian operator
with zero-mean Z; it compares it with the CT run on real data without
saying how the expectations were evaluated):
  * expectations are taken empirically on the actual phantom: the input side
    uses x = V mu_true (the preconditioned-domain signal the denoiser
    estimates) and one seeded standard-normal field v; the output side uses
    the actual line integrals z = A mu_true and counts y, with
    P = z + sqrt(tau_p) n for one seeded standard-normal field n, so that
    z - P has the variance tau_p the channel assumes;
  * -E[d g_out / dp] is, per ray, (1 - Var[z | P, y, tau_p] / tau_p) / tau_p,
    the channel's own tau_s term; the recursion uses Algorithm 1's
    normalisation: tau_p = ||Phi~||_F^2 tau_x / M, tau_r = N / (||Phi~||_F^2
    tau_s) (the printed tau_p = beta tau_x with beta = M/N contradicts it);
  * A_in carries the factor tau_r: tau_x = tau_r * mean divergence, as in
    Algorithm 1 step 4 (the printed A_in omits it); the divergence is the
    same one-probe Monte-Carlo estimate (eq. MC_SURE) at R;
  * the same damping as the algorithm is applied to tau_s and tau_x (eta = 1
    is the undamped recursion); E_in predicts the MSE of the denoiser's
    output D(r^t) before the damping mixes it with x^t.

``state_evolution`` takes the output and input maps as functions, so the
same recursion serves the CT channel and denoisers and, as its pin, an
AWGN channel with a Bernoulli-Gaussian MMSE denoiser on an i.i.d. Gaussian
operator, where it must reproduce the closed-form scalar recursion
(``gamp.se_recursion``).

Parity: pinned by that reduction (the i.i.d. case against quadrature-based
state evolution); the CT instance is unpinned against the paper (its data
and its SE figure's values are not available).
"""
import math

import numpy as np

from . import channel as _channel
from . import denoisers as _den


def state_evolution(T, fro2, M, N, tau_s_fn, denoise_fn, x_true, v, tau_x0=1.0, eta_x=1.0,
                    eta_s=1.0):
    """The scalar recursion.  tau_s_fn(tau_p, t) -> the output side's tau_s;
    denoise_fn(R, tau_r, t) -> (D(R), divergence).  Returns one record per
    iteration: tau_p, tau_s, tau_r, div, tau_x and mse_pred = E_in."""
    x_true = np.asarray(x_true, dtype=np.float64).ravel()
    v = np.asarray(v, dtype=np.float64).ravel()
    tau_x = float(tau_x0)
    tau_s = 0.0
    out = []
    for t in range(T):
        tau_p = fro2 / M * tau_x
        ts_new = tau_s_fn(tau_p, t)
        tau_s = ts_new if t == 0 else eta_s * ts_new + (1.0 - eta_s) * tau_s
        if not (math.isfinite(tau_s) and tau_s > 0):
            break
        tau_r = N / (fro2 * tau_s)
        xi_r = tau_r  # matched output channel, eq. SE_matches
        R = x_true + math.sqrt(xi_r) * v
        D, div = denoise_fn(R, tau_r, t)
        mse_pred = float(np.mean((np.asarray(D).ravel() - x_true) ** 2))
        tx_new = tau_r * div if div > 0 else 1e-12 * tau_r
        tau_x = tx_new if t == 0 else eta_x * tx_new + (1.0 - eta_x) * tau_x
        out.append(dict(t=t, tau_p=tau_p, tau_s=tau_s, tau_r=tau_r, div=div, tau_x=tau_x,
                        mse_pred=mse_pred))
        if not (math.isfinite(tau_x) and tau_x > 0):
            break
    return out


def ct_state_evolution(I, z, x_true, y, i0, fro2, T, den_kind, den_params, probe_seed, n, v,
                       eps_rel=1e-3, channel_kind=_channel.LAPLACE, tau_x0=1.0, eta_x=1.0,
                       eta_s=1.0):
    """The recursion on the CT problem: z = A mu_true (M values), x_true =
    V mu_true (I x I), y the counts; n (M values) and v (N values) are the
    standard-normal fields of the output and input sides."""
    N = I * I
    z = np.asarray(z, dtype=np.float64).ravel()
    M = z.size
    y = np.asarray(y, dtype=np.float64).ravel()
    n = np.asarray(n, dtype=np.float64).ravel()

    def tau_s_fn(tau_p, t):
        P = z + math.sqrt(tau_p) * n
        return _channel.poisson_out(P, y, tau_p, i0, channel_kind)[1]

    def denoise_fn(R, tau_r, t):
        R2 = R.reshape(I, I)
        D = _den.apply(den_kind, R2, tau_r, den_params)
        div, _ = _den.mc_divergence(den_kind, R2, tau_r, den_params, D, probe_seed, t, eps_rel)
        return D.ravel(), div

    return state_evolution(T, fro2, M, N, tau_s_fn, denoise_fn, x_true, v, tau_x0, eta_x, eta_s)
