"""Fourier-slice Radon operator, FP64 (test infrastructure).

Sec. 2.4, eq. Radon_op: A = F_gamma^-1 Omega F -- the 2D Fourier transform
of the image, sampled on a polar grid (Omega: Cartesian to polar), then a 1D
inverse Fourier transform along every radial line gives the sinogram (the
central slice theorem, eq. Acontinous).  The paper computes Omega F with a
non-uniform FFT (Kaiser-Bessel interpolation); the oracle evaluates the
polar samples exactly, as the non-uniform DFT of the image samples, so the
GPU's interpolation error is what a comparison measures.

Readings (the paper gives the operator in matrix form, without scales or
sample positions):
  * the image is the set of point masses h^2 mu_ij at the pixel centres of
    the grid of the ray-driven operator, (x_j, y_i) = ((j - (I-1)/2) h,
    ((I-1)/2 - i) h); its transform at frequency (u, v) in cycles/mm is
        P(u, v) = h^2 sum_ij mu_ij exp(-2 pi i (u x_j + v y_i));
  * view k samples the line (u, v) = rho (cos theta_k, sin theta_k), with the
    parallel geometry's theta_k, at N_dec radial frequencies
        rho_m = (m - floor(N_dec / 2)) / (N_dec d),  m = 0 .. N_dec - 1,
    d the detector pitch: the frequencies a length-N_dec DFT of the view's
    N_dec bins resolves;
  * the 1D inverse transform returns the view at the bin centres
    s_b = (b - (N_dec - 1)/2) d:
        sino_k(b) = Re (1 / (N_dec d)) sum_m P_k(m) exp(+2 pi i rho_m s_b),
    the real part (the imaginary part is zero for odd N_dec, whose rho grid
    is symmetric, and the conjugate-symmetry argument of Sec. 2.4 keeps
    the operator real).
With these scales a unit pixel at the origin projects to h at the central
bin of every view (for d = h), and every view carries the image's mass:
d sum_b sino_k(b) = h^2 sum mu.

The adjoint applies the transposed steps in reverse order (a real sinogram
in, the forward DFT along each view with the conjugate phases, then the
adjoint non-uniform DFT onto the pixel centres, real part).

Library primitives: numpy complex matrix products for the sums.

Parity: pinned (mass conservation per view, a unit pixel at the origin,
projections of a shifted Gaussian blob against its closed-form line
integral, the adjoint identity).
"""
import math

import numpy as np


def polar_frequencies(g):
    """(u, v) of every polar sample, arrays of shape (n_views, n_bins), and rho."""
    nv, nb, d = g["n_views"], g["n_bins"], g["bin_mm"]
    rho = (np.arange(nb) - nb // 2) / (nb * d)
    th = g["angle0_rad"] + np.arange(nv) * g["span_rad"] / nv
    return np.outer(np.cos(th), rho), np.outer(np.sin(th), rho), rho


def _centres(g):
    I, h = g["n"], g["pixel_mm"]
    c = (np.arange(I) - 0.5 * (I - 1)) * h
    return c, -c  # x_j for columns j, y_i for rows i


def polar_transform(mu, g):
    """P_k(m) = h^2 sum_ij mu_ij exp(-2 pi i (u x_j + v y_i)) at every polar sample."""
    mu = np.asarray(mu, dtype=np.float64)
    u, v, _ = polar_frequencies(g)
    xs, ys = _centres(g)
    h2 = g["pixel_mm"] ** 2
    U, V = u.ravel(), v.ravel()
    Ex = np.exp(-2j * math.pi * np.outer(U, xs))   # (M, I): columns
    Ey = np.exp(-2j * math.pi * np.outer(V, ys))   # (M, I): rows
    # sum_i sum_j Ey[m, i] mu[i, j] Ex[m, j]
    P = np.einsum("mi,mi->m", Ey @ mu, Ex, optimize=True) * h2
    return P.reshape(u.shape)


def radial_inverse(P, g):
    """sino_k(b) = (1 / (N_dec d)) sum_m P_k(m) exp(+2 pi i rho_m s_b), complex."""
    nb, d = g["n_bins"], g["bin_mm"]
    _, _, rho = polar_frequencies(g)
    s = (np.arange(nb) - 0.5 * (nb - 1)) * d
    E = np.exp(2j * math.pi * np.outer(rho, s))    # (m, b)
    return (P @ E) / (nb * d)


def project(mu, g):
    """The Fourier-slice projection of mu, real, shape (n_views, n_bins)."""
    return np.real(radial_inverse(polar_transform(mu, g), g))


def backproject(sino, g):
    """The adjoint of ``project`` (real sinogram in, real image out)."""
    nb, d = g["n_bins"], g["bin_mm"]
    _, _, rho = polar_frequencies(g)
    s = (np.arange(nb) - 0.5 * (nb - 1)) * d
    E = np.exp(-2j * math.pi * np.outer(s, rho))   # (b, m): conjugate of radial_inverse
    Q = (np.asarray(sino, dtype=np.float64) @ E) / (nb * d)
    u, v, _ = polar_frequencies(g)
    xs, ys = _centres(g)
    h2 = g["pixel_mm"] ** 2
    Ex = np.exp(2j * math.pi * np.outer(u.ravel(), xs))
    Ey = np.exp(2j * math.pi * np.outer(v.ravel(), ys))
    # out[i, j] = h^2 Re sum_m Q_m Ey[m, i] Ex[m, j]
    out = (Ey * Q.ravel()[:, None]).T @ Ex
    return np.real(out) * h2
