"""Pins of the oracle's Fourier-slice Radon operator (Sec. 2.4, eq. Radon_op)."""
import math

import numpy as np

from oracle import fourier
from paper_1609_04661_amd import synth


def _g(I=32, nv=12, nb=47, h=1.0, d=1.0, a0=0.1):
    return synth.geometry(synth.PARALLEL, I, h, nv, nb, math.pi, angle0_rad=a0, bin_mm=d)


def test_every_view_carries_the_mass():
    rng = np.random.default_rng(0)
    for g in (_g(), _g(I=20, nv=7, nb=32, h=0.5, d=0.7)):
        mu = rng.random((g["n"], g["n"]))
        z = fourier.project(mu, g)
        assert np.allclose(z.sum(axis=1) * g["bin_mm"], g["pixel_mm"] ** 2 * mu.sum(), rtol=1e-12)


def test_unit_pixel_at_origin():
    # odd I: pixel (I//2, I//2) sits at the origin; its transform is h^2 at every frequency,
    # so with d = h every view reads h at the central bin (odd N_dec) and the rest of the
    # Dirichlet kernel elsewhere
    g = _g(I=15, nv=5, nb=21)
    mu = np.zeros((15, 15))
    mu[7, 7] = 1.0
    z = fourier.project(mu, g)
    assert np.allclose(z[:, 10], 1.0, atol=1e-12)
    assert np.allclose(z[:, :10], 0.0, atol=1e-12) and np.allclose(z[:, 11:], 0.0, atol=1e-12)


def test_shifted_gaussian_matches_its_line_integrals():
    # a smooth blob exp(-|p - c|^2 / (2 s^2)) has line integrals sqrt(2 pi) s exp(-(t - t0)^2 /
    # (2 s^2)) with t0 = <c, n_theta>; the point-mass model converges to them while the blob
    # is well sampled and inside the band; a sign slip in any phase moves the peak to -t0
    I, h, s = 64, 1.0, 3.0
    c = np.array([7.5, -4.25])
    g = _g(I=I, nv=9, nb=91, h=h, d=1.0, a0=0.3)
    xs = (np.arange(I) - 0.5 * (I - 1)) * h
    X, Y = np.meshgrid(xs, -xs, indexing="xy")
    mu = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * s * s))
    z = fourier.project(mu, g)
    th = g["angle0_rad"] + np.arange(9) * math.pi / 9
    t = (np.arange(91) - 45.0) * 1.0
    t0 = c[0] * np.cos(th) + c[1] * np.sin(th)
    ref = math.sqrt(2 * math.pi) * s * np.exp(-(t[None, :] - t0[:, None]) ** 2 / (2 * s * s))
    assert np.max(np.abs(z - ref)) < 1e-6 * ref.max()


def test_adjoint_identity():
    rng = np.random.default_rng(1)
    for g in (_g(), _g(I=24, nv=10, nb=36, h=0.8, d=1.1)):
        mu = rng.standard_normal((g["n"], g["n"]))
        sv = rng.standard_normal((g["n_views"], g["n_bins"]))
        lhs = float(np.sum(fourier.project(mu, g) * sv))
        rhs = float(np.sum(mu * fourier.backproject(sv, g)))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
