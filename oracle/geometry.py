"""Ray lines of the two acquisition geometries, in FP64 (test infrastructure).

Sec. 2.1 (eq. linCT, eq. Phi_mtx): the system matrix has one row per ray,
J = N_dec * N_theta rows, rows ordered view-major (ray index = k*N_dec + b);
sparse-view sub-selection S is implicit: only the measured views exist.

Each ray is returned as the line {u : <u, n> = s} with unit normal
n = (cos theta, sin theta) and signed offset s (mm).

Conventions (the paper gives none; Sec. 6 names a fan geometry, the configs
name parallel and fan):
  * parallel: theta_k = angle0 + k*span/N_theta (end point excluded),
    s_b = (b - (N_dec-1)/2) * bin_mm;
  * fan (equiangular arc detector): source S_k = D_so (cos beta_k, sin beta_k),
    beta_k = angle0 + k*span/N_theta, ray b leaves S_k towards the
    iso-centre rotated by gamma_b = (b - (N_dec-1)/2) * dgamma.  Its line has
    normal angle beta_k + gamma_b + pi/2 and offset -D_so sin(gamma_b).
    dgamma = 0 selects the pitch that makes the fan cover the circle that
    circumscribes the image: 2 asin(I h / (sqrt(2) D_so)) / N_dec;
  * angles that are exact multiples of pi/2 use exact trig values (0, +-1),
    so grid-aligned rays lie exactly on pixel edges.

Parity: pinned indirectly by the chord tests of ``radon`` (closed-form chords
of single pixels and of the whole grid for every ray).
"""
import math

import numpy as np

PARALLEL = 0
FAN = 1


def snapped_cos_sin(theta):
    """cos/sin with exact values at multiples of pi/2."""
    q = theta / (0.5 * math.pi)
    k = round(q)
    if abs(q - k) < 1e-12:
        return [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][k % 4]
    return math.cos(theta), math.sin(theta)


def fan_dgamma(g):
    if g.get("dgamma_rad", 0.0):
        return g["dgamma_rad"]
    R = g["n"] * g["pixel_mm"] / math.sqrt(2.0)
    return 2.0 * math.asin(R / g["dso_mm"]) / g["n_bins"]


def ray_lines(g):
    """Return (nx, ny, s) FP64 arrays of length n_views * n_bins."""
    nv, nb = g["n_views"], g["n_bins"]
    nx = np.empty(nv * nb)
    ny = np.empty(nv * nb)
    s = np.empty(nv * nb)
    c0 = 0.5 * (nb - 1)
    if g["kind"] == PARALLEL:
        for k in range(nv):
            th = g["angle0_rad"] + k * g["span_rad"] / nv
            c, sn = snapped_cos_sin(th)
            for b in range(nb):
                r = k * nb + b
                nx[r], ny[r] = c, sn
                s[r] = (b - c0) * g["bin_mm"]
    elif g["kind"] == FAN:
        dg = fan_dgamma(g)
        for k in range(nv):
            beta = g["angle0_rad"] + k * g["span_rad"] / nv
            for b in range(nb):
                gam = (b - c0) * dg
                c, sn = snapped_cos_sin(beta + gam + 0.5 * math.pi)
                r = k * nb + b
                nx[r], ny[r] = c, sn
                s[r] = -g["dso_mm"] * math.sin(gam)
    else:
        raise ValueError("unknown geometry kind")
    return nx, ny, s
