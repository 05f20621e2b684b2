"""Pins of the oracle's scalar state evolution (Sec. 4.4, eqs. SEasym,
SE_matches, E_in, A_in): on an i.i.d. Gaussian operator with an AWGN output
channel and the Bernoulli-Gaussian MMSE denoiser, the recursion evaluated
empirically on a large sample must reproduce the quadrature-based scalar
recursion E_{t+1} = mmse(sw2 + (N/M) E_t); a mis-scaled step fails it."""
import math

import numpy as np

from oracle import gamp, se

RHO, SX2, SW2 = 0.1, 1.0, 1e-3
N, M, T = 2000, 1000, 8
NS = 200000  # sample size of the empirical expectations


def _iid_se(xi_scale=1.0, fro2_scale=1.0):
    rng = np.random.default_rng(11)
    x = (rng.random(NS) < RHO) * rng.normal(0, math.sqrt(SX2), NS)
    v = rng.standard_normal(NS)
    den = gamp.bg_denoiser(RHO, SX2)
    fro2 = float(N) * fro2_scale  # ||Phi||_F^2 of an N(0, 1/M) matrix with N columns

    def tau_s_fn(tau_p, t):
        return 1.0 / (tau_p + SW2)

    def denoise_fn(R, tau_r, t):
        # a planted mis-scaling of the input noise (xi_r != tau_r) enters here
        Rp = x + math.sqrt(xi_scale) * (R - x)
        return den(Rp, tau_r, t)

    return se.state_evolution(T, fro2, M, N, tau_s_fn, denoise_fn, x, v, tau_x0=RHO * SX2)


def test_state_evolution_reduces_to_the_iid_recursion():
    recs = _iid_se()
    ref = gamp.se_recursion(RHO, SX2, SW2, N / M, T, RHO * SX2)[1:]
    pred = np.array([r["mse_pred"] for r in recs])
    assert np.all(np.abs(pred - ref) / ref < 0.03), (pred, ref)
    # matched MMSE denoiser: tau_x (posterior variance) equals the predicted MSE
    tx = np.array([r["tau_x"] for r in recs])
    assert np.all(np.abs(tx - pred) / pred < 0.03)
    # and tau_r is sw2 + (N/M) tau_x of the previous step
    for a, b in zip(recs[:-1], recs[1:]):
        assert abs(b["tau_r"] - (SW2 + N / M * a["tau_x"])) < 1e-12 * b["tau_r"]


def test_planted_mistakes_break_the_reduction():
    ref = np.array(gamp.se_recursion(RHO, SX2, SW2, N / M, T, RHO * SX2)[1:])
    for kw in (dict(xi_scale=2.0), dict(fro2_scale=0.5)):
        pred = np.array([r["mse_pred"] for r in _iid_se(**kw)])
        assert np.max(np.abs(pred - ref) / ref) > 0.1, kw
