"""Exact-chord system matrix A and its transpose, FP64 (test infrastructure).

Sec. 2.1, eqs. paramdiscrete / linCT: with pixel indicator basis functions
b_j, a_ij is the length of ray L_i inside pixel j, z = A mu sums
chord * mu_j along each ray, and A^T uses the same weights, so the adjoint
is exact.  The chords come from the C core (``oracle_line_segments``), which
intersects each line with every grid line, sorts the crossings and assigns
each segment to the pixel holding its midpoint; a line lying on a pixel edge
gives half of its length to each neighbour.

Parity: pinned (closed-form chords of single pixels and of the full grid,
the adjoint identity, convergence to analytic ellipse line integrals).
"""
import numpy as np

from . import _lib
from .geometry import ray_lines


class Radon:
    def __init__(self, g):
        self.g = dict(g)
        self.I = g["n"]
        self.h = g["pixel_mm"]
        self.nx, self.ny, self.s = ray_lines(g)
        self.M = self.nx.size
        self.N = self.I * self.I

    def project(self, img):
        img = np.ascontiguousarray(img, dtype=np.float64).reshape(self.N)
        out = np.empty(self.M)
        _lib.lib().oracle_project(self.I, self.h, self.M, _lib.dptr(self.nx), _lib.dptr(self.ny),
                                  _lib.dptr(self.s), _lib.dptr(img), _lib.dptr(out))
        return out.reshape(self.g["n_views"], self.g["n_bins"])

    def backproject(self, sino):
        sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(self.M)
        out = np.empty(self.N)
        _lib.lib().oracle_backproject(self.I, self.h, self.M, _lib.dptr(self.nx), _lib.dptr(self.ny),
                                      _lib.dptr(self.s), _lib.dptr(sino), _lib.dptr(out))
        return out.reshape(self.I, self.I)

    def line_segments(self, r):
        """(pixel index, chord length) pairs of ray r."""
        cap = 8 * self.I + 32
        idx = np.zeros(cap, dtype=np.int32)
        ln = np.zeros(cap)
        lam = np.zeros(2 * self.I + 8)
        m = _lib.lib().oracle_line_segments(self.I, self.h, float(self.nx[r]), float(self.ny[r]),
                                            float(self.s[r]), _lib.iptr(idx), _lib.dptr(ln),
                                            _lib.dptr(lam))
        return idx[:m].copy(), ln[:m].copy()

    def dense(self):
        """Dense M x N matrix (small grids only)."""
        A = np.zeros((self.M, self.N))
        for r in range(self.M):
            idx, ln = self.line_segments(r)
            np.add.at(A[r], idx, ln)
        return A
