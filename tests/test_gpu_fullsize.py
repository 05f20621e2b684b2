"""Configured full-size D-GAMP-CT runs through the C ABI against stored FP64
oracle results (``tests/golden/*.npz``, written by ``tests/golden/make_golden.py``,
which calls only the oracle and the seeded input generators).

Cases:
  * c2: the headline workload -- 512 x 512, 64 parallel views x 729 bins,
    I0 = 1e5, NLM, damping 0.15, all 50 iterations;
  * c3: the first 384 x 384 slice of the uneven batch (its own view count and
    I0), 30 iterations, run as one slice of a two-slice batch (the batch path
    the uneven workload uses) and on its own;
  * c5: slice 0 of the fan-beam low-dose batch (1024 x 1024 at 0.5 mm, 128
    views over 360 deg, 1024 bins, I0 = 5e3), NLM, 3 iterations.

Tolerances:
  * PSNR within 0.1 dB of the oracle's (the accuracy target);
  * mu relative L2 (over the stored pixels: all of them, or every second row
    and column at 1024 x 1024) within 3x the oracle's own sensitivity: the stored
    distance between the oracle's run and the same run with every iterate x
    multiplied by (1 + 2e-5 xi), xi a +-1 field per iteration.  2e-5 is the
    denoiser's per-call FP32 parity bound (the largest per-iteration error of
    the GPU kernels), so the sensitivity is how far the recursion carries
    errors of that size; the factor 3 allows for their being correlated
    rather than random in sign.  A floor of 1e-4 covers cases where the
    recursion damps them below the FP32 resolution of the final V^-1;
  * the first iteration's tau_p, tau_s, tau_r (no denoiser error yet: FP64
    reductions of FP32 terms): relative 1e-5.
"""
import importlib.util
import json
import os

import numpy as np
import pytest
import torch

from oracle import metrics, radon
from paper_1609_04661_amd import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)


def load_case(name):
    z = np.load(os.path.join(HERE, "golden", name + ".npz"), allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    c = golden.CASES[name]()
    R = radon.Radon(c["geom"])
    y = synth.poisson_counts(R.project(c["mu"]), c["i0"], c["seed"])
    # the same counts the oracle's run was given
    assert float(y.sum()) == float(z["y_sum"]) and float((y * y).sum()) == float(z["y_sq"])
    assert meta["T"] == c["T"] and meta["eta"] == c["eta"]
    return c, y, z


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def check(c, z, mu_gpu, log_gpu, status):
    assert status == 0.0
    psnr_gpu = metrics.psnr(mu_gpu, c["mu"])
    psnr_ref = float(z["psnr"])
    ref = z["mu_hat"].astype(np.float64)
    k = json.loads(str(z["meta"])).get("stride", 1)  # stored every k-th row and column
    got = mu_gpu[::k, ::k]
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    bound = max(3.0 * float(z["sens_rel"]), 1e-4)
    print("psnr gpu %.4f oracle %.4f | mu rel %.3e (bound %.3e)" % (psnr_gpu, psnr_ref, rel, bound))
    assert abs(psnr_gpu - psnr_ref) <= 0.1, (psnr_gpu, psnr_ref)
    assert rel <= bound, (rel, bound)
    L = z["log"]
    for k in range(3):  # tau_p, tau_s, tau_r
        assert abs(log_gpu[0, k] - L[0, k]) <= 1e-5 * abs(L[0, k]), (k, log_gpu[0, k], L[0, k])


def run_single(api, c, y, fro2):
    P = api.Plan(c["geom"])
    T = c["T"]
    st = api.DgampState(P, 1.0)
    mu = torch.empty((P.I, P.I), dtype=torch.float32, device="cuda")
    log = torch.zeros(T * api.LOG_STRIDE, dtype=torch.float64, device="cuda")
    api.dgamp_iterate(P, torch.as_tensor(y, dtype=torch.float32).cuda(), st, T, fro2, c["i0"],
                      api.DEN_NLM, api.make_params(api.DEN_NLM), probe_seed=c["probe_seed"],
                      eta_x=c["eta"], eta_s=c["eta"], mu_out=mu, log=log)
    return host(mu), host(log).reshape(T, api.LOG_STRIDE), float(host(st.scal)[api.S_STATUS])


@pytest.mark.parametrize("name", ["c2", "c5"])
def test_fullsize_run_matches_oracle(gpu_lib, name):
    c, y, z = load_case(name)
    mu, log, status = run_single(gpu_lib, c, y, float(z["fro2"]))
    check(c, z, mu, log, status)


def test_c3_slice_in_batch_matches_oracle(gpu_lib):
    """The 384 x 384 slice as slice 1 of a batch whose slice 0 is a 256 x 256,
    32-view slice (the batch's per-phase launches cover both), and on its own."""
    api = gpu_lib
    c, y, z = load_case("c3")
    fro2 = float(z["fro2"])
    mu1, log1, st1 = run_single(api, c, y, fro2)
    check(c, z, mu1, log1, st1)
    g0 = synth.geometry(synth.PARALLEL, 256, 1.0, 32, 363, np.pi)
    mu0 = synth.ellipse_phantom(256, 77)
    P0 = api.Plan(g0)
    y0 = synth.poisson_counts(radon.Radon(g0).project(mu0), 2e4, 77)
    fro2_0 = float(api.dg_fro2_hutchinson(P0, 8, 99).item())
    B = api.Batch([g0, c["geom"]])
    yb = torch.cat([torch.as_tensor(y0, dtype=torch.float32).reshape(-1),
                    torch.as_tensor(y, dtype=torch.float32).reshape(-1)]).cuda().contiguous()
    mu_out = torch.empty(B.totN, dtype=torch.float32, device="cuda")
    B.bind(yb, [2e4, c["i0"]], [fro2_0, fro2], api.DEN_NLM, api.make_params(api.DEN_NLM), mu_out)
    B.state_init(1.0)
    B.iterate(c["T"], probe_seed=c["probe_seed"], eta_x=c["eta"], eta_s=c["eta"], write_mu=True)
    mub = host(B.image(mu_out, 1)).reshape(mu1.shape)
    # slice 1 of the batch is the single-slice run, bit for bit
    assert np.array_equal(mub, mu1)
    assert float(host(B.scal[api.NSCAL + api.S_STATUS:api.NSCAL + api.S_STATUS + 1])[0]) == 0.0


def test_check_status_reports_undamped_divergence(gpu_lib):
    """Algorithm 1 undamped on the headline inputs stops with a non-finite or
    non-positive variance; the synchronous status check returns DG_ERR_NUMERIC
    naming the iteration the device status word recorded, and DG_OK for the
    damped run."""
    api = gpu_lib
    c, y, z = load_case("c2")
    P = api.Plan(c["geom"])
    yd = torch.as_tensor(y, dtype=torch.float32).cuda()
    for eta, T in ((1.0, 30), (0.15, 5)):
        st = api.DgampState(P, 1.0)
        api.dgamp_iterate(P, yd, st, T, float(z["fro2"]), c["i0"], api.DEN_NLM,
                          api.make_params(api.DEN_NLM), probe_seed=7, eta_x=eta, eta_s=eta)
        rc, fs, fi = api.dg_check_status(st.scal)
        status = float(host(st.scal)[api.S_STATUS])
        if eta == 1.0:
            assert status > 0 and rc == api.ERR_NUMERIC and fs == 0 and fi == int(status) - 1
        else:
            assert status == 0 and rc == 0 and fs == -1 and fi == -1


def test_learned_denoiser_gains_over_plain(gpu_lib):
    """The shipped CNN weights against the plain patch-based denoiser on the
    headline inputs (same counts, probes, damping 0.15, 50 iterations): the
    learned run ends at least 0.5 dB higher and reaches the plain run's final
    PSNR in at most 40 of the 50 iterations."""
    import os
    api = gpu_lib
    c, y, z = load_case("c2")
    P = api.Plan(c["geom"])
    yd = torch.as_tensor(y, dtype=torch.float32).cuda()
    mu_true = torch.as_tensor(c["mu"], dtype=torch.float32).cuda()
    weights = os.path.join(os.path.dirname(HERE), "paper_1609_04661_amd", "weights",
                           "cnn_c2_x_space.safetensors")
    net = api.CnnNet.load_file(weights)
    runs = {"plain": (api.DEN_NLM, api.make_params(api.DEN_NLM)),
            "learned": (api.DEN_CNN, api.make_params(api.DEN_CNN, net=net, n_pixels=P.N))}
    curves = {}
    mu = torch.empty((P.I, P.I), dtype=torch.float32, device="cuda")
    for name, (kind, prm) in runs.items():
        st = api.DgampState(P, 1.0)
        ps = torch.empty(c["T"], dtype=torch.float64, device="cuda")
        for t in range(c["T"]):
            api.dgamp_iterate(P, yd, st, 1, float(z["fro2"]), c["i0"], kind, prm, probe_seed=7,
                              eta_x=c["eta"], eta_s=c["eta"], mu_out=mu)
            api.dg_psnr(mu, mu_true, out=ps[t:t + 1])
        curves[name] = host(ps)
        assert float(host(st.scal)[api.S_STATUS]) == 0.0
    plain, learned = curves["plain"], curves["learned"]
    reach = int(np.argmax(learned >= plain[-1])) + 1 if np.any(learned >= plain[-1]) else None
    print("final psnr plain %.3f learned %.3f; learned reaches plain's final at iteration %s"
          % (plain[-1], learned[-1], reach))
    assert abs(plain[-1] - float(z["psnr"])) <= 0.1
    assert learned[-1] >= plain[-1] + 0.5 and reach is not None and reach <= 40
