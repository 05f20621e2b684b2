"""dgamp_iterate_noalloc (no workspace argument, no device allocation) against
dgamp_iterate on the same inputs, through the C ABI: two calls in a row, the
second with a smaller image, must give bit-identical states, scalars, logs and
mu (the two entry points launch the same kernels; only where the iteration
workspace lives differs), and a plan whose workspace exceeds the fixed
scratch array is refused with nothing launched."""
import math

import numpy as np
import pytest
import torch

from paper_1609_04661_amd import synth

pytestmark = pytest.mark.gpu


def inputs(api, g, i0, seed):
    P = api.Plan(g)
    mu = torch.as_tensor(synth.ellipse_phantom(g["n"], seed, pixel_mm=g["pixel_mm"]),
                         dtype=torch.float32).cuda()
    z = api.ct_project(P, mu)
    torch.cuda.synchronize()
    y = torch.as_tensor(synth.poisson_counts(z.cpu().double().numpy(), i0, seed),
                        dtype=torch.float32).cuda()
    fro2 = float(api.dg_fro2_hutchinson(P, 4, 99).item())
    return P, y, fro2


def run(api, P, y, fro2, i0, T, noalloc):
    st = api.DgampState(P, 1.0)
    mu = torch.empty((P.I, P.I), dtype=torch.float32, device="cuda")
    log = torch.zeros(T * api.LOG_STRIDE, dtype=torch.float64, device="cuda")
    kw = dict(probe_seed=21, eta_x=0.5, eta_s=0.5, mu_out=mu, log=log)
    params = api.make_params(api.DEN_NLM)
    if noalloc:
        api.dgamp_iterate_noalloc(P, y, st, T, fro2, i0, api.DEN_NLM, params, **kw)
    else:
        api.dgamp_iterate(P, y, st, T, fro2, i0, api.DEN_NLM, params, **kw)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (st.x, st.s, st.scal, mu, log)]


def test_noalloc_matches_dgamp_iterate(gpu_lib):
    api = gpu_lib
    big = synth.geometry(synth.PARALLEL, 256, 1.0, 48, 363, math.pi)
    small = synth.c1_geometry()
    for g, i0, T in ((big, 3e4, 4), (small, 1e4, 3)):
        P, y, fro2 = inputs(api, g, i0, 5)
        assert int(api.load().dg_workspace_bytes(P.handle, api.OP_DGAMP)) <= api.dg_noalloc_scratch_bytes()
        ref = run(api, P, y, fro2, i0, T, noalloc=False)
        got = run(api, P, y, fro2, i0, T, noalloc=True)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        assert ref[2][api.S_STATUS] == 0.0


def test_noalloc_refuses_plans_beyond_its_scratch(gpu_lib):
    api = gpu_lib
    g = synth.geometry(synth.PARALLEL, 2048, 1.0, 2, 2897, math.pi)
    P = api.Plan(g)
    assert int(api.load().dg_workspace_bytes(P.handle, api.OP_DGAMP)) > api.dg_noalloc_scratch_bytes()
    st = api.DgampState(P, 1.0)
    y = torch.ones(P.M, dtype=torch.float32, device="cuda")
    with pytest.raises(api.DgError, match="scratch"):
        api.dgamp_iterate_noalloc(P, y, st, 1, 1.0, 1e4, api.DEN_NLM, api.make_params(api.DEN_NLM))
