"""Fourier-slice Radon operator (Sec. 2.4, eq. Radon_op) through the C ABI
against the oracle's exact evaluation (the non-uniform DFT on the polar grid
and the direct radial inverse DFT, FP64).  The GPU interpolates with a
Kaiser-Bessel kernel of width 8 on a 2x oversampled grid (relative error
~1.5e-8 in FP64) and computes in FP32: a 2D FFT of side 2I and a direct
radial DFT of n_bins terms each carry relative errors of ~eps32 log2(2I) and
~eps32 sqrt(n_bins) ~ 1e-6, so the projection bound of the ray-driven
operator, 1e-5 relative L2, applies; every element within 1e-4 of the
largest.  The adjoint: the same bounds against the oracle's adjoint, and
the GPU adjoint identity to 1e-5."""
import math

import numpy as np
import pytest
import torch

from oracle import fourier
from paper_1609_04661_amd import synth

pytestmark = pytest.mark.gpu

GEOMS = {
    "c1": synth.c1_geometry(),
    "even_bins": synth.geometry(synth.PARALLEL, 128, 0.8, 40, 180, math.pi, angle0_rad=0.3, bin_mm=0.9),
    "c2": synth.c2_geometry(),
}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


@pytest.mark.parametrize("name", list(GEOMS))
def test_fourier_project_and_adjoint_match_oracle(gpu_lib, name):
    api = gpu_lib
    g = GEOMS[name]
    op = api.FourierOp(g)
    mu = synth.ellipse_phantom(g["n"], 21, pixel_mm=g["pixel_mm"]).astype(np.float32).astype(np.float64)
    z = api.ct_project_fourier(op, cu(mu))
    torch.cuda.synchronize()
    z = z.cpu().double().numpy()
    ref = fourier.project(mu, g)
    print(name, "project rel %.2e max %.2e" % (rel(z, ref), np.max(np.abs(z - ref)) / np.max(np.abs(ref))))
    assert rel(z, ref) <= 1e-5 and np.max(np.abs(z - ref)) <= 1e-4 * np.max(np.abs(ref))
    s = np.random.default_rng(3).standard_normal((g["n_views"], g["n_bins"])).astype(np.float32).astype(np.float64)
    b = api.ct_backproject_fourier(op, cu(s))
    torch.cuda.synchronize()
    b = b.cpu().double().numpy()
    bref = fourier.backproject(s, g)
    print(name, "adjoint rel %.2e" % rel(b, bref))
    assert rel(b, bref) <= 1e-5 and np.max(np.abs(b - bref)) <= 1e-4 * np.max(np.abs(bref))
    # adjoint identity on the GPU's own pair
    lhs = float(np.sum(z * s))
    rhs = float(np.sum(mu * b))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(z) * np.linalg.norm(s)


def test_fourier_rejects_unsupported_geometries(gpu_lib):
    api = gpu_lib
    for g in (synth.c5_geometry(), synth.geometry(synth.PARALLEL, 96, 1.0, 8, 137, math.pi),
              synth.geometry(synth.PARALLEL, 1024, 1.0, 8, 1449, math.pi)):
        with pytest.raises(api.DgError):
            api.FourierOp(g)
