"""Scalar state evolution (Sec. 4.4) through the C ABI against the FP64 oracle
on the same inputs (z = A mu, x = V mu, counts, the two noise fields, all
FP32-rounded before either side sees them).

Tolerance, per iteration t and per logged scalar (tau_p, tau_s, tau_r, div,
tau_x, E_in): relative 3 sum_{s <= t} e_s + 1e-5, with e_s the divergence
bound of iteration s relative to its divergence (``div_tol`` of the parity
tests at the oracle's R and D(R)).  The divergence estimate is the only
FP32 error of note in the recursion (the channel's tau_s and E_in are FP64
sums of FP32 terms, ~1e-6); it enters tau_x at its relative size, and
tau_p, tau_s, tau_r and the next input noise level follow tau_x with a
sensitivity of about one, so the errors of the iterations add up.
"""
import math

import numpy as np
import pytest
import torch

from oracle import denoisers as oden
from oracle import gamp as ogamp
from oracle import precond, radon, se
from paper_1609_04661_amd import synth
from test_gpu_parity import div_tol

pytestmark = pytest.mark.gpu

KEYS = ("tau_p", "tau_s", "tau_r", "div", "tau_x", "mse_pred")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def cu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


CASES = {
    # C1: 64 x 64, 30 views, Haar, damping 0.5, 10 iterations (and undamped, 4)
    "c1_haar": dict(geom=synth.c1_geometry(), seed=1001, i0=1e4, kind=oden.HAAR,
                    params=dict(alpha=1.5), T=10, eta=0.5, fro2="exact"),
    "c1_haar_undamped": dict(geom=synth.c1_geometry(), seed=1001, i0=1e4, kind=oden.HAAR,
                             params=dict(alpha=1.5), T=4, eta=1.0, fro2="exact"),
    # C2: 512 x 512, 64 views, NLM, damping 0.15, 5 iterations
    "c2_nlm": dict(geom=synth.c2_geometry(), seed=1002, i0=1e5, kind=oden.NLM, params={}, T=5,
                   eta=0.15, fro2="hutchinson"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_state_evolution_matches_oracle(gpu_lib, name):
    api = gpu_lib
    c = CASES[name]
    g = c["geom"]
    I = g["n"]
    R = radon.Radon(g)
    mu = synth.ellipse_phantom(I, c["seed"])
    z = f32(R.project(mu).ravel())
    x = f32(precond.apply_V(mu).ravel())
    y = synth.poisson_counts(z, c["i0"], c["seed"])
    rng = np.random.default_rng(c["seed"] + 7)
    n = f32(rng.standard_normal(z.size))
    v = f32(rng.standard_normal(x.size))
    fro2 = ogamp.fro2_exact_dense(R.dense(), I) if c["fro2"] == "exact" else ogamp.fro2_hutchinson(R, 8, 99)
    ref = se.ct_state_evolution(I, z, x, y, c["i0"], fro2, c["T"], c["kind"], c["params"], 17, n, v,
                                eta_x=c["eta"], eta_s=c["eta"])
    P = api.Plan(g)
    kind = {oden.HAAR: api.DEN_HAAR, oden.NLM: api.DEN_NLM}[c["kind"]]
    prm = api.make_params(kind, **c["params"])
    log = api.dgamp_state_evolution(P, cu(z), cu(x), cu(y), cu(n), cu(v), c["T"], fro2, c["i0"],
                                    kind, prm, probe_seed=17, eta_x=c["eta"], eta_s=c["eta"])
    torch.cuda.synchronize()
    L = log.cpu().numpy().reshape(-1, api.LOG_STRIDE)
    assert len(ref) == c["T"] and np.all(L[:, 6] == 0)
    acc = 0.0
    rho = 1e-5 if c["kind"] == oden.HAAR else 2e-5
    for t, rec in enumerate(ref):
        Rt = x + math.sqrt(rec["tau_r"]) * v
        Dt = oden.apply(c["kind"], Rt.reshape(I, I), rec["tau_r"], c["params"])
        acc += div_tol(rec["div"], Dt, Rt.reshape(I, I), rho) / abs(rec["div"])
        tol = 3 * acc + 1e-5
        got = dict(zip(KEYS, (L[t, 0], L[t, 1], L[t, 2], L[t, 3], L[t, 4], L[t, api.SE_LOG_MSE])))
        for k in KEYS:
            err = abs(got[k] - rec[k]) / abs(rec[k])
            print("t %d %-8s gpu %.9e oracle %.9e rel %.2e tol %.2e" % (t, k, got[k], rec[k], err, tol))
            assert err <= tol, (t, k, got[k], rec[k], tol)
