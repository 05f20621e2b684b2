"""BM3D plug-in denoiser through the C ABI against the oracle on the same FP32
inputs.  Both take the same decisions (block matches, surviving coefficients:
FP32 arithmetic in one fixed order on both sides), so what remains is the
FP32 arithmetic of the continuous part -- 8-point transforms, the Haar
pyramid over at most 16 blocks, the Wiener factors and the aggregation by
atomics, each a few roundings deep: relative L2 <= 1e-5 (the Haar
denoiser's bound, the same depth of transforms).  A decision taken
differently would move whole coefficients of 2.7 sigma and fail it by
orders of magnitude.  The divergence: ``div_tol`` with that rho.  D-GAMP-CT
with BM3D on C1 against the oracle's run: PSNR within 0.1 dB (the GPU's r
differs from the oracle's by FP32 rounding, so a coefficient within
rounding of its threshold may be decided differently along the way)."""
import math

import numpy as np
import pytest
import torch

from oracle import bm3d as obm3d
from oracle import denoisers as oden
from oracle import gamp as ogamp
from oracle import metrics, precond, radon
from paper_1609_04661_amd import synth
from test_gpu_parity import div_tol

pytestmark = pytest.mark.gpu


def cu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


@pytest.mark.parametrize("I,noise,tau", [(64, 0.05, 2.5e-3), (100, 0.05, 2.5e-3), (256, 0.15, 0.0225)])
def test_bm3d_matches_oracle(gpu_lib, I, noise, tau):
    api = gpu_lib
    g = synth.geometry(synth.PARALLEL, I, 1.0, 4, I + 1, math.pi)
    P = api.Plan(g)
    base = precond.apply_V(synth.ellipse_phantom(I, 6)) if I == 256 else synth.ellipse_phantom(I, 6) * 20
    r32 = (base + noise * np.random.default_rng(2).standard_normal((I, I))).astype(np.float32)
    prm = api.make_params(api.DEN_BM3D, side=I)
    x, div = api.denoise(P, api.DEN_BM3D, prm, cu(r32), torch.tensor([tau], dtype=torch.float64).cuda(),
                         probe_seed=5, iteration=1)
    torch.cuda.synchronize()
    x = x.cpu().double().numpy()
    ref = obm3d.bm3d(r32, tau)
    rel = float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
    div_ref, _ = obm3d.mc_divergence(r32, tau, ref, 5, 1)
    got = float(div.item())
    tol = div_tol(div_ref, ref, r32.astype(np.float64), 1e-5)
    print("bm3d %d rel %.2e div gpu %.7f oracle %.7f tol %.1e" % (I, rel, got, div_ref, tol))
    assert rel <= 1e-5, rel
    assert abs(got - div_ref) <= tol, (got, div_ref, tol)


def test_dgamp_c1_bm3d_matches_oracle(gpu_lib):
    api = gpu_lib
    g = synth.c1_geometry()
    R = radon.Radon(g)
    mu = synth.ellipse_phantom(64, 1001)
    y = synth.poisson_counts(R.project(mu), 1e4, 1001)
    fro2 = ogamp.fro2_exact_dense(R.dense(), 64)
    T, eta, seed = 10, 0.5, 13
    ref_mu, ref_log, _ = ogamp.dgamp_ct(R, y, 1e4, fro2, T, oden.BM3D, {}, seed, eta_x=eta, eta_s=eta)
    P = api.Plan(g)
    st = api.DgampState(P, 1.0)
    out = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    api.dgamp_iterate(P, cu(y), st, T, fro2, 1e4, api.DEN_BM3D, api.make_params(api.DEN_BM3D, side=64),
                      probe_seed=seed, eta_x=eta, eta_s=eta, mu_out=out)
    torch.cuda.synchronize()
    got = out.cpu().double().numpy()
    assert float(st.scal[api.S_STATUS].item()) == 0.0
    p_ref, p_gpu = metrics.psnr(ref_mu, mu), metrics.psnr(got, mu)
    print("dgamp bm3d psnr gpu %.4f oracle %.4f" % (p_gpu, p_ref))
    assert abs(p_gpu - p_ref) <= 0.1
