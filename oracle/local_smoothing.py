"""Geometric local smoothing (Section 2.1; Algorithms 1-2, local-smoothing
branch) (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Levels.  Multigrid level l consists of every cell of refinement level l,
refined or not.  These cells all have the same size and form a conforming mesh
of the region Omega_l that they cover, so the level space V_l (continuous Q_k
on them, zero on the domain boundary) has no hanging nodes.  Level 0 is the
coarse grid and covers the whole domain.

Refinement edge.  Where Omega_l does not reach the domain boundary, its
boundary is an internal interface.  The level-l DoFs on it are the edge DoFs
x_E; the others are the interior DoFs x_S.  The level matrix splits into the
blocks A_SS, A_SE, A_ES, A_EE (Section 2.1).  Smoothing uses A_SS only
(homogeneous Dirichlet values on the edge).  The residual handed to the
coarser level is b_S - A_SS x_S on interior DoFs and -A_ES x_S on edge DoFs
(Eq. (eq:multigrid:ls:edge): the edge part of b was already given to the
coarser level when b was copied to the levels).  Before postsmoothing the
right-hand side becomes b_S - A_SE x_E, with x_E the prolongated coarse values
(inhomogeneous Dirichlet values from the coarser level).

Copy to and from the levels (Algorithm 1).  A free DoF of the active mesh
belongs to the coarsest level among the leaves that have it as a node; there
it is an interior DoF of the level.  copy_to_mg writes each free DoF's value
into that level (all other level entries are zero) and copy_from_mg reads it
back from there.

Transfers between levels l-1 and l are the nodal injection of the level-(l-1)
function into V_l on the cells of level l (every such cell is a child of a
level-(l-1) cell); restriction is the transpose.
"""
from __future__ import annotations

import numpy as np

from . import fe, octree, solvers
from .hierarchy import degree_sequence
from .octree import _unpack3, pack
from .space import CellCoefficient, Space, assemble_stiffness, prolongation


class _LevelIndex:
    """Membership of the cells of one refinement level (the interface that
    ``space.prolongation`` uses to locate the parent of a fine cell)."""

    def __init__(self, level, keys):
        self.level = level
        self.keys = keys

    def is_leaf(self, l, i, j, k):
        return l == self.level and ((i << 42) | (j << 21) | k) in self.keys


class LevelSpace(Space):
    """Q_k on all cells of refinement level ``level`` of ``tree``; Dirichlet
    nodes on the domain boundary only; ``edge[i]`` flags refinement-edge DoFs."""

    def __init__(self, tree, level, k, coef=None):
        self.tree = tree
        self.coef = CellCoefficient(coef, tree) if coef is not None else None
        self.geometry = None  # local-smoothing levels are built on cubes
        self.level = int(level)
        self.k = int(k)
        self.n = self.k + 1
        self.dirichlet = True
        self.xi = fe.gll_points(self.k)
        self._v1d, self._rows, self._cls = {}, {}, {}
        ex = tree.existing(self.level)
        self._exists = set(ex.tolist())
        self.index = _LevelIndex(self.level, self._exists)
        self.cells = [(self.level, i, j, m) for i, j, m in _unpack3(ex).tolist()]
        self._number()
        self.edge = self._edge_flags()

    def _classify(self, cell, a, b, c):
        if self._on_boundary(cell, (a, b, c)):
            return ("dir",)
        return ("free", self.node_code(cell, a, b, c))

    def _cells_around(self, cell, abc):
        """Level-l cells (inside the domain) whose closure contains the node."""
        l, *ijk = cell
        ext = self.tree.extent(l)
        axes = []
        for idx, a in zip(ijk, abc):
            cand = [idx - 1, idx] if a == 0 else [idx, idx + 1] if a == self.k else [idx]
            axes.append([x for x in cand if 0 <= x < ext])
        return [(i, j, m) for i in axes[0] for j in axes[1] for m in axes[2]]

    def _edge_flags(self):
        """A free node lies on the refinement edge when a level-l cell around it
        does not exist (the point is covered by a coarser leaf there)."""
        edge = np.zeros(self.n_dofs, bool)
        n = self.n
        for cell in self.cells:
            rows = self.cell_rows(cell)
            q = 0
            for c in range(n):
                for b in range(n):
                    for a in range(n):
                        row = rows[q]
                        q += 1
                        if not row:
                            continue
                        g = self.key_index[row[0][0]]
                        if edge[g]:
                            continue
                        for i, j, m in self._cells_around(cell, (a, b, c)):
                            if int(pack(i, j, m)) not in self._exists:
                                edge[g] = True
                                break
        return edge


def level_numbers(tree):
    """Refinement levels that hold cells, coarse to fine (0, 1, ..., L)."""
    return [l for l in range(tree.n_levels() + 1) if tree.existing(l).size]


def copy_maps(active, spaces):
    """Per level, (level DoF indices, active DoF indices) of the free active
    DoFs that belong to the level (coarsest leaf that has the DoF as a node)."""
    owner = {}
    for cell in active.cells:
        for row in active.cell_rows(cell):
            if len(row) == 1 and row[0][1] == 1.0:
                key = row[0][0]
                owner[key] = min(owner.get(key, cell[0]), cell[0])
    maps = []
    by_level = {V.level: V for V in spaces}
    per = {V.level: ([], []) for V in spaces}
    for key, l in owner.items():
        V = by_level[l]
        j = V.key_index[key]
        assert not V.edge[j], "an active DoF is an edge DoF of its own level"
        per[l][0].append(j)
        per[l][1].append(active.key_index[key])
    for V in spaces:
        lv, ac = per[V.level]
        maps.append((np.array(lv, dtype=np.int64), np.array(ac, dtype=np.int64)))
    return maps


class LSLevel:
    """Level matrix with its interior/edge split and the A_SS smoother."""

    def __init__(self, space, P, degree):
        self.space = space
        self.A_full = assemble_stiffness(space).tocsr()
        edge = getattr(space, "edge", np.zeros(space.n_dofs, bool))  # polynomial levels: no edge
        self.S = np.flatnonzero(~edge)
        self.E = np.flatnonzero(edge)
        self.smoother = solvers.Level(self.A_full[self.S][:, self.S], None, degree)
        self.A_ES = self.A_full[self.E][:, self.S]
        self.A_SE = self.A_full[self.S][:, self.E]
        self.P = P
        self.n = space.n_dofs


class LSHierarchy:
    """Local-smoothing multigrid for the Q_k problem on the leaves of ``tree``.

    With ``coarse_p`` the coarse grid at degree k is followed by polynomial
    levels on the coarse grid, k -> floor(k/2) -> ... -> 1 (Section 2.3), and
    the direct solve happens at degree 1; these levels cover the domain and
    have no refinement edge and no share of the copied right-hand side.
    """

    def __init__(self, tree, k, cheb_degree=3, coarse_p=False, coef=None):
        self.active = Space(tree, k, coef=coef)
        self.A = assemble_stiffness(self.active)
        self.spaces = [LevelSpace(tree, l, k, coef) for l in level_numbers(tree)]
        if coarse_p:
            grid = octree.gc_sequence(tree)[-1]
            self.spaces = [Space(grid, d, coef=coef, coef_fine=tree) for d in degree_sequence(k)[:0:-1]] + self.spaces
        self.levels = []
        for l, V in enumerate(self.spaces):
            P = prolongation(V, self.spaces[l - 1]) if l > 0 else None
            self.levels.append(LSLevel(V, P, cheb_degree))
        assert self.levels[0].E.size == 0, "the coarse grid covers the domain"
        for L in self.levels[1:]:
            L.smoother.setup_smoother()
        self.coarse = solvers.CoarseDirect(self.levels[0].A_full)
        ls_spaces = [V for V in self.spaces if isinstance(V, LevelSpace)]
        ls_maps = dict(zip([V.level for V in ls_spaces], copy_maps(self.active, ls_spaces)))
        empty = (np.zeros(0, np.int64), np.zeros(0, np.int64))
        self.maps = [ls_maps[V.level] if isinstance(V, LevelSpace) else empty for V in self.spaces]

    # -- Algorithm 1 -----------------------------------------------------------------
    def copy_to_mg(self, b):
        out = []
        for L, (lv, ac) in zip(self.levels, self.maps):
            v = np.zeros(L.n)
            v[lv] = b[ac]
            out.append(v)
        return out

    def copy_from_mg(self, xs):
        x = np.zeros(self.active.n_dofs)
        for (lv, ac), xl in zip(self.maps, xs):
            x[ac] = xl[lv]
        return x

    # -- Algorithm 2, local-smoothing branch ------------------------------------------
    def vcycle_levels(self, bs):
        bs = [b.copy() for b in bs]
        xs = [None] * len(self.levels)

        def level(l):
            if l == 0:
                xs[0] = self.coarse(bs[0])
                return
            L = self.levels[l]
            sm = L.smoother
            bS = bs[l][L.S]
            xS = solvers.chebyshev(sm.A, sm.Dinv, bS, None, sm.degree, sm.lmin, sm.lmax)  # presmoothing
            r = np.zeros(L.n)
            r[L.S] = bS - sm.A @ xS                                       # residual, interior
            r[L.E] = -(L.A_ES @ xS)                                       # residual, edge
            bs[l - 1] = bs[l - 1] + L.P.T @ r                             # restriction
            level(l - 1)
            x = np.zeros(L.n)
            x[L.S] = xS
            x = x + L.P @ xs[l - 1]                                       # prolongation
            bS = bS - L.A_SE @ x[L.E]                                     # edge
            x[L.S] = solvers.chebyshev(sm.A, sm.Dinv, bS, x[L.S], sm.degree, sm.lmin, sm.lmax)  # postsmoothing
            xs[l] = x

        level(len(self.levels) - 1)
        return xs

    def vcycle(self, b):
        return self.copy_from_mg(self.vcycle_levels(self.copy_to_mg(b)))

    def solve(self, b, rtol=1e-10, max_it=200, flexible=False):
        return solvers.pcg(self.A, b, self.vcycle, rtol, max_it, flexible)
