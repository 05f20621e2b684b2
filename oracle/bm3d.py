"""Two-stage BM3D plug-in denoiser, FP64 with FP32 decisions (test infrastructure).

The paper's denoiser (Sec. 4.3 treats D as a black box; Sec. 6 and its
tables use BM3D, Dabov, Foi, Katkovnik & Egiazarian 2007).  For an I x I
input r and noise level sigma = sqrt(tau_r):

  Stage 1 (hard thresholding).  Reference blocks of n1 x n1 = 8 x 8 pixels
  on a grid of step 3 (plus the last position, so every pixel is covered).
  Each forms a group with the blocks within +-19 pixels (a 39 x 39
  window) whose mean squared difference to it is at most tau_1 = 4.8
  sigma^2: the reference block first, then the closest others ordered by
  distance (then raster position), 16 at most, the count rounded down to a
  power of two.  The group's 3D transform (orthonormal 8 x
  8 DCT-II of every block, then the orthonormal Haar pyramid along the
  group) is hard-thresholded at 2.7 sigma; N_har coefficients survive; the
  inverse transform gives block estimates, aggregated with weight
  1 / (sigma^2 N_har) (1 when none survives) times a Kaiser window
  (beta = 2): y_basic = sum w K est / sum w K.

  Stage 2 (Wiener).  The same groups; the 3D transforms of the noisy blocks
  T_n and of the basic estimate's blocks T_b give the empirical Wiener
  shrinkage W = T_b^2 / (T_b^2 + sigma^2) applied to T_n; weight
  1 / (sigma^2 ||W||^2) (1 when every factor vanishes, the basic estimate
  being zero on the whole group -- the first stage's rule for a group
  without surviving coefficients) times the Kaiser window; the result is
  D(r).

Readings (the paper names BM3D only; the values are the normal profile of
Dabov et al. for sigma up to 40 on the 8-bit scale):
  * the 8 x 8 DCT in both stages (the original's first stage uses a
    biorthogonal spline wavelet);
  * the second stage reuses the first stage's groups (the original matches
    again on the basic estimate); every decision then depends on the input r
    alone;
  * the matching threshold scales with sigma^2: the profile's first-stage
    3000 (8-bit scale, sigma <= 40) read at sigma = 25 is 4.8 sigma^2;
    tau_r spans decades in the preconditioned domain, so a fixed value
    would not do;
  * the decisions (block distances against tau_1, coefficients against
    2.7 sigma) are taken on the FP32 input in FP32 arithmetic in a fixed
    order (``oracle_bm3d_groups`` / ``oracle_bm3d_keep`` in the C core), the
    precision of the kernels, so that both sides take the same ones; the
    thresholds are computed in FP64 from tau_r and rounded to FP32.  All
    continuous arithmetic (transforms of the kept coefficients, weights,
    aggregation, Wiener) is FP64.
  * For the Monte-Carlo divergence the perturbed input is formed in FP32:
    FP32(r) + FP32(eps) b (one rounding), the input a kernel sees.

Parity: pinned (DCT orthonormality and closed-form coefficients, the Haar
pyramid against the Haar denoiser's transform, a constant image is a fixed
point, a group of identical blocks reproduces a single block's 2D
filtering, sigma -> 0 is the identity); against the paper unpinned (it
prints no BM3D values for inputs one can reproduce).
"""
import math

import numpy as np

from . import _lib
from .probe import rademacher

N1, STEP, NS, N2 = 8, 3, 19, 16
TAU_MATCH = 4.8      # tau_1 = TAU_MATCH sigma^2
LAMBDA_3D = 2.7
KAISER_BETA = 2.0


def dct_matrix(n=N1):
    """Orthonormal DCT-II: D[u, k] = a_u cos(pi (2k + 1) u / (2n))."""
    k = np.arange(n)
    D = np.cos(np.pi * (2 * k[None, :] + 1) * k[:, None] / (2 * n))
    D[0] *= math.sqrt(1.0 / n)
    D[1:] *= math.sqrt(2.0 / n)
    return D


def haar_fwd(g):
    """Orthonormal Haar pyramid along axis 0 (length a power of two)."""
    g = np.array(g, dtype=np.float64, copy=True)
    L = g.shape[0]
    c = 1.0 / math.sqrt(2.0)
    while L > 1:
        a = (g[0:L:2] + g[1:L:2]) * c
        d = (g[0:L:2] - g[1:L:2]) * c
        g[:L // 2], g[L // 2:L] = a, d
        L //= 2
    return g


def haar_inv(g):
    g = np.array(g, dtype=np.float64, copy=True)
    n = g.shape[0]
    c = 1.0 / math.sqrt(2.0)
    L = 2
    while L <= n:
        a, d = g[:L // 2].copy(), g[L // 2:L].copy()
        g[0:L:2] = (a + d) * c
        g[1:L:2] = (a - d) * c
        L *= 2
    return g


def transform3d(blocks, D):
    return haar_fwd(np.einsum("uk,bkv,wv->buw", D, blocks, D))


def inverse3d(coef, D):
    b = haar_inv(coef)
    return np.einsum("ku,bkv,vw->buw", D, b, D)


def kaiser2d():
    k = np.kaiser(N1, KAISER_BETA)
    return np.outer(k, k)


def decisions(r32, sigma2):
    """The groups and the stage-1 keep masks, from the FP32 input."""
    L = _lib.lib()
    I = r32.shape[0]
    r32 = np.ascontiguousarray(r32, dtype=np.float32)
    axis = np.zeros(I, dtype=np.int32)
    na = L.oracle_bm3d_ref_axis(I, N1, STEP, _lib.iptr(axis))
    axis = np.ascontiguousarray(axis[:na])
    nref = na * na
    grp = np.zeros(nref * N2, dtype=np.int32)
    gsize = np.zeros(nref, dtype=np.int32)
    thr = np.float32(TAU_MATCH * sigma2)
    L.oracle_bm3d_groups(I, _lib.fptr(r32.reshape(-1)), N1, NS, N2, float(thr), na,
                         _lib.iptr(axis), _lib.iptr(grp), _lib.iptr(gsize))
    D32 = np.ascontiguousarray(dct_matrix().astype(np.float32).reshape(-1))
    keep = np.zeros(nref * N2 * N1 * N1, dtype=np.uint8)
    nkeep = np.zeros(nref, dtype=np.int32)
    thr3 = np.float32(LAMBDA_3D * math.sqrt(sigma2))
    L.oracle_bm3d_keep(I, _lib.fptr(r32.reshape(-1)), N1, N2, nref, _lib.iptr(grp),
                       _lib.iptr(gsize), _lib.fptr(D32), float(thr3), _lib.u8ptr(keep),
                       _lib.iptr(nkeep))
    return axis, grp.reshape(nref, N2), gsize, keep.reshape(nref, N2, N1, N1).astype(bool), nkeep


def _blocks(img, pos, I):
    return np.stack([img[p // I:p // I + N1, p % I:p % I + N1] for p in pos])


def _aggregate(I, groups, gsize, est_w):
    num = np.zeros((I, I))
    den = np.zeros((I, I))
    K = kaiser2d()
    for q, (est, w) in enumerate(est_w):
        for b in range(gsize[q]):
            p = groups[q, b]
            y, x = p // I, p % I
            num[y:y + N1, x:x + N1] += w * K * est[b]
            den[y:y + N1, x:x + N1] += w * K
    return num / den


def bm3d(r, tau_r):
    """D(r) for sigma^2 = tau_r (r given as FP32 values)."""
    r32 = np.asarray(r, dtype=np.float32)
    r = r32.astype(np.float64)
    I = r.shape[0]
    sigma2 = float(tau_r)
    if not sigma2 > 0.0:
        return r.copy()
    D = dct_matrix()
    _, grp, gsize, keep, nkeep = decisions(r32, sigma2)
    # stage 1
    est1 = []
    for q in range(grp.shape[0]):
        n = gsize[q]
        T = transform3d(_blocks(r, grp[q, :n], I), D)
        T[~keep[q, :n]] = 0.0
        w = 1.0 / (sigma2 * nkeep[q]) if nkeep[q] >= 1 else 1.0
        est1.append((inverse3d(T, D), w))
    yb = _aggregate(I, grp, gsize, est1)
    # stage 2
    est2 = []
    for q in range(grp.shape[0]):
        n = gsize[q]
        Tn = transform3d(_blocks(r, grp[q, :n], I), D)
        Tb = transform3d(_blocks(yb, grp[q, :n], I), D)
        W = Tb * Tb / (Tb * Tb + sigma2)
        wsq = float(np.sum(W * W))
        w = 1.0 / (sigma2 * wsq) if wsq > 0.0 else 1.0
        est2.append((inverse3d(W * Tn, D), w))
    return _aggregate(I, grp, gsize, est2)


def perturbed_input(r, eps, b):
    """FP32(r) + FP32(eps) b in FP32 (one rounding), as a kernel forms it."""
    return (np.asarray(r, dtype=np.float32) + np.float32(eps) * np.asarray(b, dtype=np.float32)
            ).astype(np.float32)


def mc_divergence(r, tau_r, x_out, seed, t, eps_rel=1e-3):
    """eq. MC_SURE with one Rademacher probe at the FP32 perturbed input."""
    r32 = np.asarray(r, dtype=np.float32)
    N = r32.size
    b = rademacher(seed, t, N).reshape(r32.shape)
    eps = max(eps_rel * float(np.max(np.abs(r32))), 1e-12)
    xp = bm3d(perturbed_input(r32, eps, b), tau_r)
    return float(np.sum(b * (xp - x_out)) / (N * eps)), eps
