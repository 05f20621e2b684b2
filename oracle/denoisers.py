"""Plug-in denoisers D_tau and their divergence, FP64 (test infrastructure).

Sec. 4.3 (eqs. rGAMP, r_input, D_in): the denoiser sees r = x + sqrt(tau_r) psi
in the preconditioned space and returns x^{t+1} = D(r); its divergence
D'(r) = (1/N) sum_i dD_i/dr_i gives tau_x^{t+1} = tau_r D'(r).
eq. MC_SURE: D'(r) ~ (1/(N eps)) b^T (D(r + eps b) - D(r)) with one probe.

Denoisers (the paper uses BM3D; the Haar and patch-based plug-ins are this
build's, the paper treats D as a black box):
  * haar_soft: orthonormal 2D Haar pyramid with J levels, soft threshold
    eta(w) = sign(w) max(|w| - lam, 0) on the detail coefficients,
    lam = alpha * sqrt(tau_r); the coarsest approximation is kept.
    Exact divergence = (#approximation coeffs + #{detail: |w| > lam}) / N.
  * nlm: non-local means (patch distance averaged over a (2pr+1)^2 patch,
    (2sr+1)^2 search window, weight exp(-max(d2 - 2 sigma^2, 0)/(hfac sigma)^2),
    sigma = sqrt(tau_r), half-sample symmetric borders), from the C core.

  * prox_tv: the proximal map of isotropic total variation (the paper's
    second plug-in family, Sec. 6 "Proximal-based TV denoiser"),
    x = argmin 1/2 ||x - r||^2 + lam TV(x), lam = alpha * sqrt(tau_r), with
    forward differences and zero difference past the last row / column,
    approximated by a fixed number K of fast gradient projection steps on
    the dual problem (Beck & Teboulle 2009): the map D is those K steps.

  * bm3d: the two-stage block-matching 3D filter (module ``bm3d``), the
    paper's own denoiser; its decisions are taken on the FP32 input.

  * prox_tv_w: the same proximal map in the (V^T V)^-1 metric (Sec. 4.3 and
    Sec. 6 name it for input in the preconditioned domain),
    x = argmin 1/2 ||x - r||^2_W + lam TV(x), W = (V^T V)^-1 = 1/c on the DFT
    grid (c the cone symbol), lam = alpha * sqrt(tau_r), approximated by K
    Chambolle-Pock primal-dual steps (Chambolle & Pock 2011) with K = lam grad,
    whose primal step is a Fourier-domain division by 1 + tau w.

Parity: haar_soft pinned (orthonormality, exact divergence by brute force);
prox_tv pinned by special cases (constant images fixed, lam -> 0 identity,
large lam -> the mean), a one-row image against an exact bounded least
squares solve of the same dual, and the primal-dual gap of converged runs;
prox_tv_w pinned by its reduction to prox_tv when W = I (two different
algorithms), constant images as fixed points, a one-row image with a
non-trivial circulant W against an exact bounded least squares solve of its
dual, and the primal-dual gap of converged runs;
nlm pinned only by special cases (constant images are fixed points; sigma->0
is the identity; symmetry under image transposition) -- against the paper it
is unpinned, the paper's BM3D being a different denoiser.
"""
import math

import numpy as np

from . import _lib
from .probe import rademacher

HAAR = 0
NLM = 1
CNN = 2
TV = 3
TVW = 4
BM3D = 5

SQ2 = math.sqrt(2.0)


def haar_levels(I):
    return max(int(round(math.log2(I))) - 2, 1)


def haar_fwd(x, J):
    """Mallat-ordered orthonormal 2D Haar coefficients of a square image."""
    c = np.array(x, dtype=np.float64, copy=True)
    n = c.shape[0]
    for _ in range(J):
        a = c[:n, :n]
        lo = (a[:, 0::2] + a[:, 1::2]) / SQ2
        hi = (a[:, 0::2] - a[:, 1::2]) / SQ2
        rows = np.concatenate([lo, hi], axis=1)
        top = (rows[0::2, :] + rows[1::2, :]) / SQ2
        bot = (rows[0::2, :] - rows[1::2, :]) / SQ2
        c[:n, :n] = np.concatenate([top, bot], axis=0)
        n //= 2
    return c


def haar_inv(c, J):
    x = np.array(c, dtype=np.float64, copy=True)
    n = x.shape[0] >> (J - 1)
    for _ in range(J):
        a = x[:n, :n]
        h = n // 2
        top, bot = a[:h, :], a[h:, :]
        rows = np.empty_like(a)
        rows[0::2, :] = (top + bot) / SQ2
        rows[1::2, :] = (top - bot) / SQ2
        lo, hi = rows[:, :h], rows[:, h:]
        out = np.empty_like(a)
        out[:, 0::2] = (lo + hi) / SQ2
        out[:, 1::2] = (lo - hi) / SQ2
        x[:n, :n] = out
        n *= 2
    return x


def haar_soft(r, tau_r, alpha=1.5, J=None):
    r = np.asarray(r, dtype=np.float64)
    I = r.shape[0]
    J = J or haar_levels(I)
    lam = alpha * math.sqrt(tau_r)
    c = haar_fwd(r, J)
    k = I >> J
    detail = np.ones_like(c, dtype=bool)
    detail[:k, :k] = False
    c[detail] = np.sign(c[detail]) * np.maximum(np.abs(c[detail]) - lam, 0.0)
    return haar_inv(c, J)


def haar_soft_exact_div(r, tau_r, alpha=1.5, J=None):
    r = np.asarray(r, dtype=np.float64)
    I = r.shape[0]
    J = J or haar_levels(I)
    lam = alpha * math.sqrt(tau_r)
    c = haar_fwd(r, J)
    k = I >> J
    detail = np.ones_like(c, dtype=bool)
    detail[:k, :k] = False
    return (k * k + np.count_nonzero(np.abs(c[detail]) > lam)) / float(I * I)


def nlm(r, tau_r, pr=2, sr=10, hfac=0.4):
    r = np.ascontiguousarray(r, dtype=np.float64)
    I = r.shape[0]
    out = np.empty_like(r)
    _lib.lib().oracle_nlm(I, _lib.dptr(r), math.sqrt(max(tau_r, 0.0)), pr, sr, hfac,
                          _lib.dptr(out))
    return out


def grad_fwd(x):
    """Forward differences (g1 down the rows, g2 along the columns), zero past
    the last row / column."""
    g1 = np.zeros_like(x)
    g2 = np.zeros_like(x)
    g1[:-1, :] = x[1:, :] - x[:-1, :]
    g2[:, :-1] = x[:, 1:] - x[:, :-1]
    return g1, g2


def grad_adj(p1, p2):
    """The adjoint of grad_fwd (minus the discrete divergence)."""
    a = np.zeros_like(p1)
    a[:-1, :] -= p1[:-1, :]
    a[1:, :] += p1[:-1, :]
    a[:, :-1] -= p2[:, :-1]
    a[:, 1:] += p2[:, :-1]
    return a


def tv_iso(x):
    g1, g2 = grad_fwd(x)
    return float(np.sum(np.sqrt(g1 * g1 + g2 * g2)))


def fgp_momentum(K):
    """beta_k = (t_k - 1) / t_{k+1}, t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
    for k = 1 .. K."""
    t, out = 1.0, []
    for _ in range(K):
        t1 = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        out.append((t - 1.0) / t1)
        t = t1
    return out


def prox_tv_lam(b, lam, K=50):
    """K fast-gradient-projection steps on the dual of
    min_x 1/2 ||x - b||^2 + lam TV(x):  with x(p) = b - lam grad^T p, the dual
    min_{|p_ij| <= 1} 1/2 ||lam grad^T p - b||^2 has gradient -lam grad x(p)
    and Lipschitz constant 8 lam^2; each step takes
        p_k = P(u_k + grad x(u_k) / (8 lam)),  u_{k+1} = p_k + beta_k (p_k - p_{k-1})
    from p_0 = u_1 = 0, P the pointwise projection onto the unit disc, and
    returns x(p_K) and p_K."""
    b = np.asarray(b, dtype=np.float64)
    p1 = np.zeros_like(b)
    p2 = np.zeros_like(b)
    if not lam > 0.0:
        return b.copy(), (p1, p2)
    u1, u2 = p1.copy(), p2.copy()
    for beta in fgp_momentum(K):
        x = b - lam * grad_adj(u1, u2)
        g1, g2 = grad_fwd(x)
        q1 = u1 + g1 / (8.0 * lam)
        q2 = u2 + g2 / (8.0 * lam)
        nrm = np.maximum(1.0, np.sqrt(q1 * q1 + q2 * q2))
        n1, n2 = q1 / nrm, q2 / nrm
        u1 = n1 + beta * (n1 - p1)
        u2 = n2 + beta * (n2 - p2)
        p1, p2 = n1, n2
    return b - lam * grad_adj(p1, p2), (p1, p2)


def prox_tv(r, tau_r, alpha=0.5, iters=50):
    lam = alpha * math.sqrt(max(tau_r, 0.0))
    return prox_tv_lam(r, lam, iters)[0]


def prox_tv_metric(b, lam, w, K=50):
    """K Chambolle-Pock steps (theta = 1) on
    min_x 1/2 (x - b)^T W (x - b) + lam TV(x),  W = F^-1 diag(w) F,
    w > 0 given on b's 2D DFT grid (numpy ordering), written as
    min_x G(x) + F(K x) with K = lam grad, F the dual of the unit-disc
    indicator, and step sizes sigma = tau = 1 / (lam sqrt 8) (||grad||^2 < 8):
        p    = P(p + sigma K xbar)                      P: pointwise unit disc
        x'   = argmin G(u) + ||u - (x - tau K^T p)||^2 / (2 tau)
             = F^-1 [(F(x - tau lam grad^T p) + tau w F b) / (1 + tau w)]
        xbar = 2 x' - x
    from x = xbar = b, p = 0.  Returns x_K and p_K."""
    b = np.asarray(b, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    p1 = np.zeros_like(b)
    p2 = np.zeros_like(b)
    if not lam > 0.0:
        return b.copy(), (p1, p2)
    tau = sigma = 1.0 / (lam * math.sqrt(8.0))
    x = b.copy()
    xbar = b.copy()
    Bh = np.fft.fft2(b)
    for _ in range(K):
        g1, g2 = grad_fwd(xbar)
        q1 = p1 + sigma * lam * g1
        q2 = p2 + sigma * lam * g2
        nrm = np.maximum(1.0, np.sqrt(q1 * q1 + q2 * q2))
        p1, p2 = q1 / nrm, q2 / nrm
        v = x - tau * lam * grad_adj(p1, p2)
        xn = np.real(np.fft.ifft2((np.fft.fft2(v) + tau * w * Bh) / (1.0 + tau * w)))
        xbar = 2.0 * xn - x
        x = xn
    return x, (p1, p2)


def metric_symbol(I, metric=0):
    """w = 1/c, the symbol of (V^T V)^-1 for the cone preconditioner (the norm
    the text names); metric = 1 gives w = c, V^T V itself (the subscript the
    paper's TV figure prints)."""
    from .precond import symbol
    return symbol(I) if metric else 1.0 / symbol(I)


def prox_tv_w(r, tau_r, alpha=1.0, iters=50, metric=0):
    lam = alpha * math.sqrt(max(tau_r, 0.0))
    r = np.asarray(r, dtype=np.float64)
    return prox_tv_metric(r, lam, metric_symbol(r.shape[-1], metric), iters)[0]


def apply(kind, r, tau_r, params):
    if kind == HAAR:
        return haar_soft(r, tau_r, **params)
    if kind == NLM:
        return nlm(r, tau_r, **params)
    if kind == CNN:
        from . import cnn
        return cnn.denoise(r, params["net"])
    if kind == TV:
        return prox_tv(r, tau_r, **params)
    if kind == TVW:
        return prox_tv_w(r, tau_r, **params)
    if kind == BM3D:
        from . import bm3d
        return bm3d.bm3d(np.asarray(r, dtype=np.float32), tau_r)
    raise ValueError("unknown denoiser kind")


def mc_divergence(kind, r, tau_r, params, x_out, seed, t, eps_rel=1e-3):
    """eq. MC_SURE with K = 1 Rademacher probe; eps = eps_rel * max|r|."""
    if kind == BM3D:
        # BM3D takes its decisions on the FP32 input: the perturbed input is formed in FP32
        from . import bm3d
        return bm3d.mc_divergence(r, tau_r, x_out, seed, t, eps_rel)
    r = np.asarray(r, dtype=np.float64)
    N = r.size
    b = rademacher(seed, t, N).reshape(r.shape)
    eps = max(eps_rel * float(np.max(np.abs(r))), 1e-12)
    x_pert = apply(kind, r + eps * b, tau_r, params)
    return float(np.sum(b * (x_pert - x_out)) / (N * eps)), eps
