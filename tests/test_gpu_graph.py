"""A captured reconstruction graph replays the eager run exactly, every time."""
import numpy as np
import pytest
import torch

from oracle import gamp as ogamp
from oracle import radon
from paper_1609_04661_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["haar", "nlm"])
def test_graph_replay_equals_eager(gpu_lib, kind):
    g = synth.c1_geometry()
    R = radon.Radon(g)
    mu = synth.ellipse_phantom(64, 1001)
    y = torch.as_tensor(synth.poisson_counts(R.project(mu), 1e4, 1001), dtype=torch.float32).cuda()
    fro2 = ogamp.fro2_hutchinson(R, 8, 5)
    plan = gpu_lib.Plan(g)
    den = gpu_lib.DEN_HAAR if kind == "haar" else gpu_lib.DEN_NLM
    params = gpu_lib.make_params(den)
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
