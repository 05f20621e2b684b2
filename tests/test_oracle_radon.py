"""Pins of the oracle's exact-chord system matrix (Sec. 2.1, eq. linCT)."""
import math

import numpy as np
import pytest

from oracle import radon
from oracle.geometry import ray_lines
from paper_1609_04661_amd import synth


def clip_chord(nx, ny, s, x0, x1, y0, y1):
    """Length of the line {<u,n> = s} inside the closed box [x0,x1] x [y0,y1]
    (Liang-Barsky slab clipping), with half weight for a line on the box edge."""
    px, py = s * nx, s * ny
    dx, dy = -ny, nx
    lo, hi = -math.inf, math.inf
    on_edge = False
    for p, d, a, b in ((px, dx, x0, x1), (py, dy, y0, y1)):
        if d == 0.0:
            if p < a or p > b:
                return 0.0
            if p == a or p == b:
                on_edge = True
        else:
            t0, t1 = (a - p) / d, (b - p) / d
            lo, hi = max(lo, min(t0, t1)), min(hi, max(t0, t1))
    L = max(0.0, hi - lo)
    return 0.5 * L if on_edge else L


def pixel_box(i, j, I, h):
    x0 = (j - I / 2) * h
    y1 = (I / 2 - i) * h
    return x0, x0 + h, y1 - h, y1


@pytest.mark.parametrize("kind", ["parallel", "fan"])
def test_every_weight_matches_box_clipping(kind):
    I, h = 12, 1.0
    if kind == "parallel":
        g = synth.geometry(synth.PARALLEL, I, h, 8, 19, math.pi)   # includes 0, 45, 90, 135 deg
    else:
        g = synth.geometry(synth.FAN, I, h, 7, 15, 2 * math.pi, dso_mm=30.0, ddo_mm=20.0)
    R = radon.Radon(g)
    A = R.dense()
    nx, ny, s = ray_lines(g)
    for r in range(R.M):
        for i in range(I):
            for j in range(I):
                ref = clip_chord(nx[r], ny[r], s[r], *pixel_box(i, j, I, h))
                assert abs(A[r, i * I + j] - ref) <= 1e-12, (r, i, j, A[r, i * I + j], ref)


def test_edge_rule_axis_aligned():
    # 0 deg view, odd bin count, even grid: every ray lies on a column edge.
    I = 8
    g = synth.geometry(synth.PARALLEL, I, 1.0, 2, 9, math.pi)
    A = radon.Radon(g).dense()
    row = A[4].reshape(I, I)          # 0 deg, s = 0: the line x = 0
    assert np.allclose(row[:, 3], 0.5) and np.allclose(row[:, 4], 0.5)
    assert np.count_nonzero(row) == 2 * I
    assert abs(A[4].sum() - I) < 1e-14


def test_all_ones_image_gives_square_chords():
    g = synth.geometry(synth.PARALLEL, 32, 0.75, 13, 47, math.pi, angle0_rad=0.1)
    R = radon.Radon(g)
    z = R.project(np.ones((32, 32))).ravel()
    half = 16 * 0.75
    ref = np.array([clip_chord(a, b, c, -half, half, -half, half)
                    for a, b, c in zip(R.nx, R.ny, R.s)])
    # rays on the outer boundary count half (edge rule)
    assert np.max(np.abs(z - ref)) <= 1e-12


@pytest.mark.parametrize("kind", ["parallel", "fan"])
def test_adjoint_identity(kind):
    rng = np.random.default_rng(3)
    if kind == "parallel":
        g = synth.geometry(synth.PARALLEL, 64, 1.0, 30, 91, math.pi)
    else:
        g = synth.geometry(synth.FAN, 64, 0.5, 40, 64, 2 * math.pi, dso_mm=60.0, ddo_mm=50.0)
    R = radon.Radon(g)
    mu = rng.standard_normal((64, 64))
    sv = rng.standard_normal((g["n_views"], g["n_bins"]))
    lhs = float(np.sum(R.project(mu) * sv))
    rhs = float(np.sum(mu * R.backproject(sv)))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.sqrt(np.sum(R.project(mu) ** 2) * np.sum(sv ** 2)))


def ellipse_projection(theta, s, cx, cy, a, b, phi, v):
    """Closed-form line integral of v * indicator(ellipse)."""
    a2 = (a * math.cos(theta - phi)) ** 2 + (b * math.sin(theta - phi)) ** 2
    sp = s - (cx * math.cos(theta) + cy * math.sin(theta))
    return 2 * v * a * b * math.sqrt(max(a2 - sp * sp, 0.0)) / a2


def test_ellipse_projections_converge_first_order():
    L = 64.0                       # physical side (mm)
    cx, cy, a, b, phi, v = 5.3, -7.1, 17.0, 9.5, 0.6, 0.02
    errs = []
    for I in (32, 64, 128):
        h = L / I
        ss = 8
        off = (np.arange(ss) + 0.5) / ss
        xs = ((np.arange(I)[:, None] + off[None, :]).ravel() - I / 2) * h
        X, Y = np.meshgrid(xs, -xs, indexing="xy")
        c, s_ = math.cos(phi), math.sin(phi)
        u = ((X - cx) * c + (Y - cy) * s_) / a
        w = (-(X - cx) * s_ + (Y - cy) * c) / b
        img = v * (u * u + w * w <= 1).reshape(I, ss, I, ss).mean(axis=(1, 3))
        g = synth.geometry(synth.PARALLEL, I, h, 9, 61, math.pi, angle0_rad=0.05, bin_mm=1.0)
        R = radon.Radon(g)
        z = R.project(img).ravel()
        ref = np.array([ellipse_projection(math.atan2(ny, nx), s, cx, cy, a, b, phi, v)
                        for nx, ny, s in zip(R.nx, R.ny, R.s)])
        errs.append(float(np.sqrt(np.mean((z - ref) ** 2))))
    slope1 = math.log2(errs[0] / errs[1])
    slope2 = math.log2(errs[1] / errs[2])
    assert errs[2] < errs[1] < errs[0]
    assert 0.5 < slope1 < 2.5 and 0.5 < slope2 < 2.5, (errs, slope1, slope2)


# Fan-beam lines built independently of ``ray_lines``: the source of view k
# sits at S_k = D_so (cos beta_k, sin beta_k); ray b leaves it along the unit
# vector towards the iso-centre, -S_k / D_so, turned counter-clockwise by
# gamma_b = (b - (N_dec - 1)/2) dgamma (equiangular arc detector; dgamma = 0
# picks the pitch whose fan just covers the circle circumscribing the image).

def _fan_rays(g):
    nv, nb = g["n_views"], g["n_bins"]
    R = g["n"] * g["pixel_mm"] / math.sqrt(2.0)
    dgam = g["dgamma_rad"] or 2.0 * math.asin(R / g["dso_mm"]) / nb
    out = []
    for k in range(nv):
        beta = g["angle0_rad"] + k * g["span_rad"] / nv
        S = np.array([g["dso_mm"] * math.cos(beta), g["dso_mm"] * math.sin(beta)])
        u = -S / g["dso_mm"]
        for b in range(nb):
            gam = (b - 0.5 * (nb - 1)) * dgam
            c, s = math.cos(gam), math.sin(gam)
            d = np.array([c * u[0] - s * u[1], s * u[0] + c * u[1]])
            out.append((S, d, gam))
    return out, dgam


FAN_PIN_GEOMS = [
    dict(n=12, pixel_mm=1.0, n_views=7, n_bins=15, span=2 * math.pi, dso=30.0, a0=0.0),
    dict(n=64, pixel_mm=0.5, n_views=9, n_bins=33, span=2 * math.pi, dso=60.0, a0=0.3),
    dict(n=1024, pixel_mm=0.5, n_views=5, n_bins=1025, span=2 * math.pi, dso=600.0, a0=0.0),
]


@pytest.mark.parametrize("p", FAN_PIN_GEOMS)
def test_fan_lines_pass_through_source_and_turn_by_gamma(p):
    g = synth.geometry(synth.FAN, p["n"], p["pixel_mm"], p["n_views"], p["n_bins"], p["span"],
                       angle0_rad=p["a0"], dso_mm=p["dso"], ddo_mm=0.5 * p["dso"])
    nx, ny, s = ray_lines(g)
    rays, dgam = _fan_rays(g)
    for r, (S, d, gam) in enumerate(rays):
        n = np.array([nx[r], ny[r]])
        assert abs(np.hypot(*n) - 1.0) < 1e-14
        # the source lies on the line, and the line runs along d
        assert abs(S @ n - s[r]) < 1e-11 * p["dso"], r
        assert abs(d @ n) < 1e-14, r
        # (the two checks above fix the sign of gamma: a ray turned by -gamma_b leaves the
        # source along the mirror of d, which is not perpendicular to n off the centre)
        # distance from the iso-centre: D_so |sin gamma|
        assert abs(abs(s[r]) - p["dso"] * abs(math.sin(gam))) < 1e-11 * p["dso"], r
    nb = p["n_bins"]
    R = p["n"] * p["pixel_mm"] / math.sqrt(2.0)
    for k in range(p["n_views"]):
        # odd bin count: the central ray passes through the iso-centre
        assert abs(s[k * nb + (nb - 1) // 2]) < 1e-12
        # the outermost rays lie half a bin inside the tangents to the circumscribed circle
        edge = p["dso"] * math.sin((nb - 1) / nb * math.asin(R / p["dso"]))
        assert abs(abs(s[k * nb]) - edge) < 1e-9 and abs(abs(s[k * nb + nb - 1]) - edge) < 1e-9


def test_fan_projection_of_off_centre_disk_matches_closed_form():
    # the line integral of a disk of radius rho at c is 2 sqrt(rho^2 - d^2), d the distance
    # from c to the ray (taken here from the independently built source and direction); the
    # pixelised disk converges to it at first order in h
    I, h, rho, v = 128, 0.5, 9.0, 0.03
    c = np.array([11.0, -6.5])
    g = synth.geometry(synth.FAN, I, h, 12, 97, 2 * math.pi, angle0_rad=0.2, dso_mm=120.0,
                       ddo_mm=80.0)
    ss = 8
    off = (np.arange(ss) + 0.5) / ss
    xs = ((np.arange(I)[:, None] + off[None, :]).ravel() - I / 2) * h
    X, Y = np.meshgrid(xs, -xs, indexing="xy")
    img = v * (((X - c[0]) ** 2 + (Y - c[1]) ** 2) <= rho * rho).reshape(I, ss, I, ss).mean(axis=(1, 3))
    z = radon.Radon(g).project(img).ravel()
    rays, _ = _fan_rays(g)
    ref = np.empty(len(rays))
    for r, (S, d, _) in enumerate(rays):
        e = c - S
        dist = abs(e[0] * d[1] - e[1] * d[0])
        ref[r] = 2.0 * v * math.sqrt(max(rho * rho - dist * dist, 0.0))
    hit = ref > 0
    assert hit.sum() > 100 and (~hit).sum() > 100
    # chord error of a staircase disk is O(h): bound by a few pixel widths of attenuation
    assert np.max(np.abs(z - ref)) < 4 * h * v
    assert np.sqrt(np.mean((z - ref) ** 2)) < 0.6 * h * v
