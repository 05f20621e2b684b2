"""Pins of the oracle's cone preconditioner (Sec. 2.4, eqs. PPFT preconditioner, Aprecon, GramATA)."""
import math

import numpy as np
import pytest

from oracle import precond, radon
from paper_1609_04661_amd import synth


@pytest.mark.parametrize("I", [16, 24, 64])
def test_single_fourier_mode_closed_form(I):
    # V^-1 multiplies the mode (kx, ky) by sqrt(|k| / I) (|rho| in cycles per pixel).
    ii, jj = np.meshgrid(np.arange(I), np.arange(I), indexing="ij")
    for kx, ky in [(1, 0), (0, 3), (2, 5), (I // 2, 0), (I // 2, I // 2), (-3, 4)]:
        wave = np.cos(2 * math.pi * (kx * jj + ky * ii) / I)
        gain = math.sqrt(math.hypot(kx, ky) / I)
        assert np.max(np.abs(precond.apply_Vinv(wave) - gain * wave)) < 1e-12
        assert np.max(np.abs(precond.apply_V(wave) - wave / gain)) < 1e-11


def test_dc_value():
    I = 32
    one = np.ones((I, I))
    # mean of 1/|rho| over the central cell [-1/(2I), 1/(2I)]^2, checked by quadrature
    from scipy import integrate
    a = 1.0 / (2 * I)
    quarter = integrate.dblquad(lambda y, x: 1.0 / math.hypot(x, y), 0, a, 0, a,
                                epsabs=1e-12, epsrel=1e-10)[0]
    val = 4 * quarter / (2 * a) ** 2
    assert abs(val - precond.DC_FACTOR * I) < 1e-6 * val
    assert np.allclose(precond.apply_Vinv(one), one / math.sqrt(val), rtol=1e-6)


def test_inverse_pair_and_symmetry():
    rng = np.random.default_rng(0)
    for I in (24, 64):
        u, w = rng.standard_normal((2, I, I))
        assert np.max(np.abs(precond.apply_V(precond.apply_Vinv(u)) - u)) < 1e-12
        assert np.max(np.abs(precond.apply_Vinv(precond.apply_V(u)) - u)) < 1e-12
        a = np.sum(precond.apply_Vinv(u) * w)
        b = np.sum(u * precond.apply_Vinv(w))
        assert abs(a - b) < 1e-12 * np.sqrt(np.sum(u * u) * np.sum(w * w))


def test_symbol_real_even():
    c = precond.symbol(24)
    k = np.arange(24)
    flip = c[np.ix_((-k) % 24, (-k) % 24)]
    assert np.array_equal(c, flip) and np.all(c > 0)


def test_preconditioning_flattens_gram_spectrum():
    # eq. GramATA: A~^T A~ is close to a multiple of I; A^T A is not.
    I = 32
    g = synth.geometry(synth.PARALLEL, I, 1.0, 50, 47, math.pi)   # ~ pi I / 2 views
    A = radon.Radon(g).dense()
    At = np.stack([precond.apply_Vinv(r.reshape(I, I)).ravel() for r in A])
    sa = np.linalg.svd(A, compute_uv=False)
    st = np.linalg.svd(At, compute_uv=False)
    # condition number of the Gram (ratio of extreme eigenvalues) on the full-rank part
    ka = (sa[0] / sa[-1]) ** 2
    kt = (st[0] / st[-1]) ** 2
    assert kt < ka / 10, (ka, kt)
    # and the bulk of the spectrum narrows (1st..99th percentile spread)
    spread = lambda v: np.percentile(v, 99) / np.percentile(v, 1)
    assert spread(st) < spread(sa) / 1.5, (spread(sa), spread(st))
