"""Cone preconditioner V = F^-1 C^(1/2) F and its inverse, FP64 (test infrastructure).

Sec. 2.4, eq. PPFT preconditioner: C = diag(1/|rho|) on the 2D DFT grid,
|rho| = sqrt(a^2 + b^2); eq. Aprecon: A~ = A V^-1 = ... C^(-1/2) F, so V^-1
multiplies the spectrum by |rho|^(1/2) (the "cone" high-pass) and V by
|rho|^(-1/2).  eq. GramATA: A~^T A~ is (approximately) the identity.

Readings (the paper is silent or singular here):
  * F is the unitary 2D DFT on the unpadded I x I grid, so V is circulant
    and V V^-1 = I exactly (the change of coordinates x = V mu of eq.
    precondAMP needs an exact inverse);
  * |rho| is measured in cycles per pixel: c(k) = I / sqrt(kx^2 + ky^2) for
    integer DFT indices k != 0;
  * the DC value, infinite in the paper, is the mean of 1/|rho| over the
    central DFT cell [-1/(2I), 1/(2I)]^2, which is 4 ln(1 + sqrt 2) I.

The FFT is numpy's (a library primitive).

Parity: pinned (closed-form action on single Fourier modes, V V^-1 = I,
self-adjointness, flattening of the Gram spectrum).
"""
import math

import numpy as np

DC_FACTOR = 4.0 * math.log(1.0 + math.sqrt(2.0))


def symbol(I):
    """c(k) = 1/|rho_k| on the DFT grid (numpy fft ordering), FP64."""
    k = np.fft.fftfreq(I) * I
    ky, kx = np.meshgrid(k, k, indexing="ij")
    rho = np.sqrt(kx * kx + ky * ky)
    c = np.empty_like(rho)
    nz = rho > 0
    c[nz] = I / rho[nz]
    c[~nz] = DC_FACTOR * I
    return c


def _filter(img, power):
    img = np.asarray(img, dtype=np.float64)
    I = img.shape[-1]
    H = symbol(I) ** power
    return np.real(np.fft.ifft2(np.fft.fft2(img) * H))


def apply_Vinv(x):
    """mu = V^-1 x (cone high-pass, multiplies the spectrum by c^(-1/2))."""
    return _filter(x, -0.5)


def apply_V(mu):
    """x = V mu (multiplies the spectrum by c^(+1/2))."""
    return _filter(mu, 0.5)
