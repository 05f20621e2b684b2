"""Seeded synthetic inputs: phantoms, acquisition parameters, Poisson counts.

This module holds none of the reconstruction method's arithmetic.  It draws
the synthetic stand-ins for the paper's data (Sec. 6: a 512 x 512 abdomen
slice, sparse views, I0 of 1e4 / 1e5; Sec. 7: cargo scans), which are not
available here:

  * ellipse phantoms: additive ellipses (semi-axes 2..20 px at 64 x 64,
    scaled with the image side), rotation U[0, pi), attenuation U[0, 0.05]/mm,
    bounding circle inside the inscribed field-of-view disk, pixel values from
    4 x 4 super-sampling;
  * for sides >= 256, Gaussian-textured regions on odd-indexed ellipses:
    white noise smoothed with a 1.5 px Gaussian, scaled to std 0.002/mm,
    masked by the ellipse;
  * optional small high-attenuation inserts (radius U[1, 4] mm,
    U[0.2, 0.5]/mm);
  * Poisson counts y ~ Poisson(I0 exp(-z)) for given line integrals z.  The
    caller supplies z (the reconstruction library's own projector, or any
    other), so no projector lives here.

Everything is drawn from numpy's PCG64 generator at an explicit seed.
"""
import math

import numpy as np

PARALLEL = 0
FAN = 1


def geometry(kind, n, pixel_mm, n_views, n_bins, span_rad, angle0_rad=0.0, bin_mm=None,
             dso_mm=0.0, ddo_mm=0.0, dgamma_rad=0.0):
    """Plain parameter record of one acquisition (no arithmetic)."""
    return dict(kind=kind, n=int(n), pixel_mm=float(pixel_mm), n_views=int(n_views),
                n_bins=int(n_bins), angle0_rad=float(angle0_rad), span_rad=float(span_rad),
                bin_mm=float(pixel_mm if bin_mm is None else bin_mm), dso_mm=float(dso_mm),
                ddo_mm=float(ddo_mm), dgamma_rad=float(dgamma_rad))


def _ellipse_mask_ss(n, cx, cy, a, b, phi, ss=4):
    """Area fraction of each pixel inside an ellipse (centre/axes in pixel units)."""
    # pixel (i, j) covers [j, j+1] x [i, i+1] in (column, row) coordinates
    off = (np.arange(ss) + 0.5) / ss
    r0 = max(int(math.floor(cy - max(a, b))) - 1, 0)
    r1 = min(int(math.ceil(cy + max(a, b))) + 1, n)
    c0 = max(int(math.floor(cx - max(a, b))) - 1, 0)
    c1 = min(int(math.ceil(cx + max(a, b))) + 1, n)
    frac = np.zeros((n, n))
    if r1 <= r0 or c1 <= c0:
        return frac
    rows = (np.arange(r0, r1)[:, None] + off[None, :]).ravel()
    cols = (np.arange(c0, c1)[:, None] + off[None, :]).ravel()
    Y, X = np.meshgrid(rows, cols, indexing="ij")
    dx, dy = X - cx, Y - cy
    c, s = math.cos(phi), math.sin(phi)
    u = (dx * c + dy * s) / a
    v = (-dx * s + dy * c) / b
    inside = (u * u + v * v <= 1.0).astype(np.float64)
    inside = inside.reshape(r1 - r0, ss, c1 - c0, ss).mean(axis=(1, 3))
    frac[r0:r1, c0:c1] = inside
    return frac


def ellipse_phantom(n, seed, n_ellipses=10, texture=None, pixel_mm=1.0, inserts=0):
    """mu (1/mm), float64 n x n, row 0 on top."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = n / 64.0
    R = n / 2.0
    img = np.zeros((n, n))
    if texture is None:
        texture = n >= 256
    for e in range(n_ellipses):
        a = rng.uniform(2.0, 20.0) * scale
        b = rng.uniform(2.0, 20.0) * scale
        phi = rng.uniform(0.0, math.pi)
        v = rng.uniform(0.0, 0.05)
        rad = max(a, b)
        room = max(R - rad, 0.0)
        rho = room * math.sqrt(rng.uniform(0.0, 1.0))
        ang = rng.uniform(0.0, 2 * math.pi)
        cx, cy = R + rho * math.cos(ang), R + rho * math.sin(ang)
        frac = _ellipse_mask_ss(n, cx, cy, a, b, phi)
        img += v * frac
        if texture and (e % 2 == 1):
            from scipy.ndimage import gaussian_filter
            w = gaussian_filter(rng.standard_normal((n, n)), 1.5)
            w *= 0.002 / max(float(np.std(w)), 1e-30)
            img += w * (frac > 0.5)
    for _ in range(int(inserts)):
        rr = rng.uniform(1.0, 4.0) / pixel_mm
        v = rng.uniform(0.2, 0.5)
        room = max(R - rr - 1.0, 0.0)
        rho = room * math.sqrt(rng.uniform(0.0, 1.0))
        ang = rng.uniform(0.0, 2 * math.pi)
        cx, cy = R + rho * math.cos(ang), R + rho * math.sin(ang)
        img += v * _ellipse_mask_ss(n, cx, cy, rr, rr, 0.0)
    return np.maximum(img, 0.0)


def poisson_counts(z, i0, seed):
    """y ~ Poisson(I0 exp(-z)), float64 (integers)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = i0 * np.exp(-np.asarray(z, dtype=np.float64))
    return rng.poisson(lam).astype(np.float64)


# ------------------------------------------------------------- named workloads

def c1_geometry():
    """64 x 64, 1 mm pixels, 30 parallel views over 180 degrees, 91 bins."""
    return geometry(PARALLEL, 64, 1.0, 30, 91, math.pi)


def c2_geometry():
    """512 x 512, 1 mm pixels, 64 parallel views over 180 degrees, 729 bins."""
    return geometry(PARALLEL, 512, 1.0, 64, 729, math.pi)


def c5_geometry():
    """1024 x 1024, 0.5 mm pixels, fan beam D_so 600 / D_od 500 mm, 128 views over 360 deg,
    1024 equiangular bins covering the circumscribed field of view."""
    return geometry(FAN, 1024, 0.5, 128, 1024, 2 * math.pi, dso_mm=600.0, ddo_mm=500.0)


def batch_slices(seed, n_slices=64):
    """Per-slice draws of the uneven batch: side in {256, 384, 512}, views in {32, 64, 128}
    over 180 degrees, bins = ceil(sqrt(2) side), I0 log-uniform in [5e3, 1e5]."""
    out = []
    for k in range(n_slices):
        rng = np.random.Generator(np.random.PCG64(seed + k))
        n = int(rng.choice([256, 384, 512]))
        nv = int(rng.choice([32, 64, 128]))
        i0 = float(math.exp(rng.uniform(math.log(5e3), math.log(1e5))))
        nb = int(math.ceil(math.sqrt(2.0) * n))
        out.append(dict(geom=geometry(PARALLEL, n, 1.0, nv, nb, math.pi), i0=i0,
                        seed=seed + k))
    return out


def c5_slices(seed, n_slices=16):
    """The fan-beam low-dose batch: every slice the C5 geometry at I0 = 5e3,
    with 1-5 high-attenuation inserts drawn per slice."""
    out = []
    for k in range(n_slices):
        rng = np.random.Generator(np.random.PCG64(seed + k))
        out.append(dict(geom=c5_geometry(), i0=5e3, seed=seed + k,
                        inserts=int(rng.integers(1, 6))))
    return out
