"""A captured reconstruction graph replays the eager run exactly, every time."""
import numpy as np
import pytest
import torch

from oracle import gamp as ogamp
from oracle import radon
from paper_1609_04661_amd import synth

pytestmark = pytest.mark.gpu


def den_params(gpu_lib, kind):
    """Denoiser kind and parameters at the 64 x 64 C1 side."""
    if kind == "haar":
        return gpu_lib.DEN_HAAR, gpu_lib.make_params(gpu_lib.DEN_HAAR)
    if kind == "nlm":
        return gpu_lib.DEN_NLM, gpu_lib.make_params(gpu_lib.DEN_NLM)
    if kind == "tv":
        return gpu_lib.DEN_TV, gpu_lib.make_params(gpu_lib.DEN_TV, n_pixels=64 * 64)
    return gpu_lib.DEN_TVW, gpu_lib.make_params(gpu_lib.DEN_TVW, side=64, alpha=1.0, iters=20,
                                                metric=1)


@pytest.mark.parametrize("kind", ["haar", "nlm", "tv", "tvw"])
def test_graph_replay_equals_eager(gpu_lib, kind):
    g = synth.c1_geometry()
    R = radon.Radon(g)
    mu = synth.ellipse_phantom(64, 1001)
    y = torch.as_tensor(synth.poisson_counts(R.project(mu), 1e4, 1001), dtype=torch.float32).cuda()
    fro2 = ogamp.fro2_hutchinson(R, 8, 5)
    plan = gpu_lib.Plan(g)
    den, params = den_params(gpu_lib, kind)
    T = 6
    # eager reference
    st = gpu_lib.DgampState(plan, 1.0)
    ref = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    gpu_lib.dgamp_iterate(plan, y, st, T, fro2, 1e4, den, params, probe_seed=9, eta_x=0.5,
                          eta_s=0.5, mu_out=ref)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    # graph
    st2 = gpu_lib.DgampState(plan, 1.0)
    out = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    graph = gpu_lib.DgampGraph(plan, y, st2, T, fro2, 1e4, den, params, tau_x0=1.0, mu_out=out,
                               probe_seed=9, eta_x=0.5, eta_s=0.5)
    for rep in range(3):
        out.fill_(float("nan"))
        junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep
        assert float(st2.scal[gpu_lib.S_STATUS].item()) == 0.0
        del junk


@pytest.mark.parametrize("kind", ["nlm", "tv", "tvw"])
def test_split_calls_equal_one_call(gpu_lib, kind):
    """T iterations in one dgamp_iterate call against T calls of one iteration
    (with and without mu_out): with NLM the divergence step's scalar finish
    is deferred into the next V^-1 x or the call's end, so the state, the log
    rows and mu must not depend on how the iterations are split."""
    g = synth.c1_geometry()
    R = radon.Radon(g)
    mu = synth.ellipse_phantom(64, 1001)
    y = torch.as_tensor(synth.poisson_counts(R.project(mu), 1e4, 1001), dtype=torch.float32).cuda()
    fro2 = ogamp.fro2_hutchinson(R, 8, 5)
    plan = gpu_lib.Plan(g)
    den, params = den_params(gpu_lib, kind)
    T = 5
    kw = dict(probe_seed=3, eta_x=0.5, eta_s=0.5)
    st1 = gpu_lib.DgampState(plan, 1.0)
    mu1 = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    log1 = torch.zeros(T * gpu_lib.LOG_STRIDE, dtype=torch.float64, device="cuda")
    gpu_lib.dgamp_iterate(plan, y, st1, T, fro2, 1e4, den, params, mu_out=mu1, log=log1, **kw)
    st2 = gpu_lib.DgampState(plan, 1.0)
    mu2 = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    log2 = torch.zeros(T * gpu_lib.LOG_STRIDE, dtype=torch.float64, device="cuda")
    for t in range(T):
        gpu_lib.dgamp_iterate(plan, y, st2, 1, fro2, 1e4, den, params,
                              mu_out=mu2 if t % 2 == 0 else None,
                              log=log2[t * gpu_lib.LOG_STRIDE:(t + 1) * gpu_lib.LOG_STRIDE], **kw)
    torch.cuda.synchronize()
    assert torch.equal(st1.x, st2.x) and torch.equal(st1.s, st2.s)
    assert torch.equal(st1.scal, st2.scal)
    assert torch.equal(log1, log2)
    assert torch.equal(mu1, mu2)
