"""Pins of the oracle's two-stage BM3D plug-in denoiser."""
import math

import numpy as np

from oracle import bm3d


def test_dct_is_orthonormal_with_closed_form_rows():
    D = bm3d.dct_matrix()
    assert np.allclose(D @ D.T, np.eye(8), atol=1e-14)
    assert np.allclose(D[0], 1 / math.sqrt(8), atol=1e-15)
    assert abs(D[1, 0] - 0.5 * math.cos(math.pi / 16)) < 1e-15


def test_haar_pyramid_closed_form_and_inverse():
    g = bm3d.haar_fwd(np.array([1.0, -1.0, 1.0, -1.0]))
    assert np.allclose(g, [0, 0, math.sqrt(2), math.sqrt(2)], atol=1e-15)
    g = bm3d.haar_fwd(np.array([1.0, 1.0, 1.0, 1.0]))
    assert np.allclose(g, [2, 0, 0, 0], atol=1e-15)
    x = np.random.default_rng(0).standard_normal((16, 3))
    assert np.allclose(bm3d.haar_inv(bm3d.haar_fwd(x)), x, atol=1e-13)
    assert abs(np.sum(bm3d.haar_fwd(x) ** 2) - np.sum(x ** 2)) < 1e-12


def test_constant_image_is_shrunk_by_the_closed_form_wiener_factor():
    # every block equals every other: full groups of 16; the only non-zero coefficient of a
    # group is its DC, 16 blocks x 8 (2D DC of an 8 x 8 block) / sqrt(16)... = 32 c, kept by
    # stage 1 (32 c > 2.7 sigma), so the basic estimate is c and stage 2 scales the DC by
    # W = (32 c)^2 / ((32 c)^2 + sigma^2): D(c) = c W everywhere
    c, s2 = 0.3, 0.01
    out = bm3d.bm3d(np.full((40, 40), c, dtype=np.float32), s2)
    c32 = float(np.float32(c))
    W = (32 * c32) ** 2 / ((32 * c32) ** 2 + s2)
    assert np.max(np.abs(out - c32 * W)) < 1e-12


def test_tiny_sigma_is_the_identity():
    r = np.random.default_rng(1).standard_normal((32, 32)).astype(np.float32)
    out = bm3d.bm3d(r, 1e-20)
    assert np.max(np.abs(out - r.astype(np.float64))) < 1e-10


def _groups_by_hand(r32, sigma2):
    """The documented matching, written out with numpy float32 scalars."""
    I = r32.shape[0]
    axis = list(range(0, I - 8 + 1, 3))
    if axis[-1] != I - 8:
        axis.append(I - 8)
    thr = np.float32(4.8 * sigma2)
    out = []
    for yr in axis:
        for xr in axis:
            cand = []
            for y in range(max(0, yr - 19), min(I - 8, yr + 19) + 1):
                for x in range(max(0, xr - 19), min(I - 8, xr + 19) + 1):
                    if (y, x) == (yr, xr):
                        continue
                    acc = np.float32(0)
                    for u in range(8):
                        for v in range(8):
                            t = np.float32(r32[yr + u, xr + v] - r32[y + u, x + v])
                            acc = np.float32(acc + np.float32(t * t))
                    d = np.float32(acc * np.float32(1 / 64))
                    if d <= thr:
                        cand.append((float(d), y * I + x))
            cand.sort()
            pos = [yr * I + xr] + [p for _, p in cand]   # the reference block leads
            take = min(len(pos), 16)
            g = 1
            while 2 * g <= take:
                g *= 2
            out.append(pos[:g])
    return out


def test_groups_follow_the_documented_matching():
    rng = np.random.default_rng(2)
    r = (np.kron(rng.random((3, 3)), np.ones((6, 6))) + 0.05 * rng.standard_normal((18, 18))).astype(np.float32)
    _, grp, gsize, _, _ = bm3d.decisions(r, 0.01)
    ref = _groups_by_hand(r, 0.01)
    assert len(ref) == grp.shape[0]
    for q, g in enumerate(ref):
        assert gsize[q] == len(g) and list(grp[q, :gsize[q]]) == g, q
    assert gsize.max() > 1 and gsize.min() >= 1


def test_bm3d_denoises_and_its_divergence_is_unbiased_in_the_mean():
    rng = np.random.default_rng(3)
    yy, xx = np.mgrid[0:48, 0:48]
    clean = (np.sin(xx / 5.0) + (yy > 20)).astype(np.float64)
    s2 = 0.04
    r = (clean + math.sqrt(s2) * rng.standard_normal(clean.shape)).astype(np.float32)
    x = bm3d.bm3d(r, s2)
    assert np.mean((x - clean) ** 2) < 0.4 * np.mean((r - clean) ** 2)
    div, eps = bm3d.mc_divergence(r, s2, x, 5, 0)
    assert 0.0 < div < 1.0


def test_group_with_vanishing_basic_estimate_gets_unit_weight():
    # zero input: every stage-1 coefficient is cut, the basic estimate is zero, every Wiener
    # factor vanishes; the defined weight keeps the output finite (and zero)
    out = bm3d.bm3d(np.zeros((24, 24), dtype=np.float32), 0.5)
    assert np.all(np.isfinite(out)) and np.max(np.abs(out)) == 0.0
