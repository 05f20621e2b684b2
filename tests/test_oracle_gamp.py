"""Pins of the oracle's GAMP recursion (Algorithm 1, Sec. 3, Sec. 4.4)."""
import math

import numpy as np
import pytest

from oracle import denoisers, gamp, metrics, radon
from paper_1609_04661_amd import synth

RHO, SX2, SW2 = 0.1, 1.0, 1e-3
N, M, T = 2000, 1000, 10


def run_iid(seed, onsager=True):
    """One GAMP run on an i.i.d. N(0, 1/M) matrix; returns per-iteration
    (actual error variance of r, the recursion's tau_r, MSE of x^{t+1})."""
    rng = np.random.default_rng(seed)
    Phi = rng.standard_normal((M, N)) / math.sqrt(M)
    x_true = (rng.random(N) < RHO) * rng.normal(0, math.sqrt(SX2), N)
    y = Phi @ x_true + rng.normal(0, math.sqrt(SW2), M)
    fro2 = float(np.sum(Phi * Phi))
    rerr, taur, mse = [], [], []
    den = gamp.bg_denoiser(RHO, SX2)

    def in_fn(r, tau_r, t):
        rerr.append(float(np.mean((r - x_true) ** 2)))
        taur.append(tau_r)
        x, d = den(r, tau_r, t)
        mse.append(float(np.mean((x - x_true) ** 2)))
        return x, d

    with np.errstate(all="ignore"):
        gamp.gamp(lambda x: Phi @ x, lambda s: Phi.T @ s, fro2, M, N, T, gamp.awgn_out(y, SW2),
                  in_fn, tau_x0=RHO * SX2, onsager=onsager)
    return np.array(rerr), np.array(taur), np.array(mse)


def test_gamp_follows_state_evolution():
    runs = [run_iid(s) for s in range(20)]
    # the recursion's tau_r is the actual error variance of r (averaged over seeds)
    calib = np.mean([re / tr for re, tr, _ in runs], axis=0)
    assert np.all(np.abs(calib[1:] - 1.0) < 0.1), calib
    # and the MSE follows the scalar state evolution E_{t+1} = mmse(sw2 + (N/M) E_t)
    se = np.array(gamp.se_recursion(RHO, SX2, SW2, N / M, T, RHO * SX2)[1:])
    emp = np.mean([ms for _, _, ms in runs], axis=0)
    assert np.all(np.abs(emp - se) / se < 0.3), (emp, se)
    assert np.all(np.abs(emp[:2] - se[:2]) / se[:2] < 0.1), (emp, se)
    assert se[-1] < 0.05 * se[0] and emp[-1] < 0.05 * emp[0]


def test_planted_onsager_removal_breaks_state_evolution():
    # the same loop without the Onsager term loses the calibration: the pin is sensitive
    runs = [run_iid(s, onsager=False) for s in range(3)]
    calib = np.mean([re / tr for re, tr, _ in runs], axis=0)
    assert np.nanmax(calib) > 3.0


def test_fro2_hutchinson_matches_exact():
    g = synth.c1_geometry()
    R = radon.Radon(g)
    exact = gamp.fro2_exact_dense(R.dense(), 64)
    K = 64
    samples = gamp.fro2_hutchinson(R, K, 1000, samples=True)
    se = np.std(samples, ddof=1) / math.sqrt(K)
    assert abs(np.mean(samples) - exact) < 3 * se


@pytest.fixture(scope="module")
def c1_case():
    g = synth.c1_geometry()
    R = radon.Radon(g)
    mu = synth.ellipse_phantom(64, 1001)
    y = synth.poisson_counts(R.project(mu), 1e4, 1001)
    fro2 = gamp.fro2_exact_dense(R.dense(), 64)
    return R, mu, y, fro2


def test_dgamp_c1_damped_improves(c1_case):
    R, mu, y, fro2 = c1_case
    ps = []
    from oracle import precond
    cb = lambda t, x, lg: ps.append(metrics.psnr(precond.apply_Vinv(x.reshape(64, 64)), mu))
    mu_hat, log, _ = gamp.dgamp_ct(R, y, 1e4, fro2, 20, denoisers.HAAR, dict(alpha=1.5), 7,
                                   eta_x=0.5, eta_s=0.5, callback=cb)
    assert ps[-1] > ps[0] + 6.0
    assert abs(ps[-1] - metrics.psnr(mu_hat, mu)) < 1e-9
    assert all(l["tau_x"] > 0 and l["tau_r"] > 0 for l in log)


def test_dgamp_c1_undamped_diverges(c1_case):
    # Algorithm 1 verbatim (no damping) does not converge on this synthetic case; this is why
    # the configured runs use the damped recursion.
    R, mu, y, fro2 = c1_case
    with np.errstate(all="ignore"):
        try:
            mu_hat, _, _ = gamp.dgamp_ct(R, y, 1e4, fro2, 20, denoisers.HAAR, dict(alpha=1.5), 7)
            bad = (not np.all(np.isfinite(mu_hat))) or metrics.psnr(mu_hat, mu) < 5.0
        except gamp.GampError:
            bad = True
    assert bad
