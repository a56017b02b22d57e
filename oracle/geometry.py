"""Mapped cell geometry (oracle): cells that are not axis-aligned cubes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The matrix-free operator of Eq. (impl:mf) applies, at every quadrature point
q of a cell, the metric term of the map x = F_e(xi) from the reference cube:
w_q |det J_q| J_q^{-1} J_q^{-T}, J_q = dx/dxi (Section 3.2).  Here that map is
built as follows.  A geometry descriptor moves the vertices of the coarse
grid; each coarse cell C becomes the trilinear (Q1) image F_C of the unit cube
through its eight moved vertices; a refined cell of level l inherits the part
of F_C over its sub-box, so F_e(xi) = F_C((r + xi) / 2^l), r the cell's
integer position inside C.  The restriction of a trilinear map to a sub-box
is again trilinear, and every level's cells tile the same deformed domain, so
the finite element spaces of the levels stay nested (the prolongation is the
same nodal injection as for cubes).

Descriptor kinds (the library's geometry kinds):

* 0: none (axis-aligned cubes).
* 1: affine, x' = M x with M = [[p0, p1, p2], [0, p3, p4], [0, 0, p5]]
  (every cell a parallelepiped).
* 2: interior bump, x' = x + p0 s(x) (p1, p2, p3) with
  s(x) = prod_d sin(pi (x_d - lo) / (hi - lo)): the boundary of the domain
  [lo, hi]^3 does not move (s = 0 there), interior vertices do, and the
  cells become general trilinear hexahedra.
"""
from __future__ import annotations

import numpy as np

# reference vertex v = a + 2b + 4c sits at (a, b, c)
_VERTS = np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=float)


def move(desc, x, lo, hi):
    """Image of points x (m, 3) under the descriptor's vertex motion."""
    kind, p = desc["kind"], list(desc["params"]) + [0.0] * 8
    x = np.atleast_2d(np.asarray(x, dtype=float))
    if kind == 0:
        return x.copy()
    if kind == 1:
        M = np.array([[p[0], p[1], p[2]], [0.0, p[3], p[4]], [0.0, 0.0, p[5]]])
        return x @ M.T
    if kind == 2:
        s = np.prod(np.sin(np.pi * (x - lo) / (hi - lo)), axis=1)
        return x + p[0] * s[:, None] * np.array(p[1:4])[None, :]
    raise ValueError(kind)


class CoarseTrilinearGeometry:
    """F_e of every cell of an octree mesh from a geometry descriptor."""

    def __init__(self, tree, desc):
        self.tree = tree
        self.desc = desc
        self.h0 = (tree.hi - tree.lo) / tree.n0

    def coarse_vertices(self, I, J, K):
        """The 8 moved vertices (8, 3) of coarse cell (I, J, K)."""
        x = self.tree.lo + self.h0 * (np.array([I, J, K], float)[None, :] + _VERTS)
        return move(self.desc, x, self.tree.lo, self.tree.hi)

    def _coarse(self, cell, xi):
        l, i, j, m = cell
        s = 2 ** l
        I, J, K = i // s, j // s, m // s
        t = (np.array([i - I * s, j - J * s, m - K * s], float)[None, :] + np.atleast_2d(xi)) / s
        return self.coarse_vertices(I, J, K), t, s

    def points(self, cell, xi):
        """x = F_e(xi) for reference points xi (m, 3)."""
        X, t, _ = self._coarse(cell, xi)
        N = np.stack([np.prod(np.where(_VERTS[v][None, :] > 0, t, 1.0 - t), axis=1) for v in range(8)], axis=1)
        return N @ X

    def jacobians(self, cell, xi):
        """J (m, 3, 3), J[q, d, e] = d x_d / d xi_e at the points xi."""
        X, t, s = self._coarse(cell, xi)
        m = t.shape[0]
        J = np.zeros((m, 3, 3))
        for v in range(8):
            f = [np.where(_VERTS[v][d] > 0, t[:, d], 1.0 - t[:, d]) for d in range(3)]
            df = [1.0 if _VERTS[v][d] > 0 else -1.0 for d in range(3)]
            grad = np.stack([df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]], axis=1)  # dN/dt
            J += X[v][None, :, None] * grad[:, None, :]
        return J / s
