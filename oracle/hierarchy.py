"""Multigrid level hierarchies (oracle).

``geometry`` (a descriptor of ``oracle.geometry``) maps the cells of every
level by the same coarse-cell trilinear maps, so the levels stay nested.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Level sequences, coarse to fine, as (mesh, degree) pairs:

* ``"h"``      geometric global coarsening (Section 2.2) at a fixed degree.
* ``"p_then_h"`` polynomial global coarsening on the finest mesh with the
  bisection rule p_c = floor(p_f / 2) (Section 2.3), then geometric global
  coarsening of the mesh at degree 1.
* ``"h_then_p"`` geometric global coarsening at the finest degree down to the
  coarse grid, then bisection of the degree on the coarse grid (used to make
  the coarse problem small enough for a direct solve).
* ``"hp"``     geometric and polynomial coarsening in the same step while both
  are possible, then the remaining one alone (the variant that the outlook,
  Section 8, leaves to future work).
"""
from __future__ import annotations

from . import octree, solvers
from .space import Space, assemble_stiffness, prolongation


def degree_sequence(k):
    seq = [k]
    while seq[-1] > 1:
        seq.append(seq[-1] // 2)
    return seq  # fine to coarse


def level_pairs(tree, k, scheme="h"):
    """(mesh, degree) pairs from coarse to fine."""
    meshes = octree.gc_sequence(tree)  # fine to coarse
    if scheme == "h":
        pairs = [(m, k) for m in meshes]
    elif scheme == "p_then_h":
        degs = degree_sequence(k)
        pairs = [(tree, d) for d in degs] + [(m, 1) for m in meshes[1:]]
    elif scheme == "h_then_p":
        degs = degree_sequence(k)
        pairs = [(m, k) for m in meshes] + [(meshes[-1], d) for d in degs[1:]]
    elif scheme == "hp":
        # mesh and degree coarsened in the same step while both can be
        degs = degree_sequence(k)
        pairs = [(meshes[min(i, len(meshes) - 1)], degs[min(i, len(degs) - 1)])
                 for i in range(max(len(meshes), len(degs)))]
    else:
        raise ValueError(scheme)
    return pairs[::-1]


class Hierarchy:
    """``drop_coarse`` leaves out that many of the coarsest levels: the direct
    coarse solve then acts on a finer level, which may have hanging nodes
    (the early switch to the coarse-grid solver of the outlook, Section 8)."""

    def __init__(self, tree, k, scheme="h", cheb_degree=3, dirichlet=True, drop_coarse=0, coef=None,
                 geometry=None):
        self.pairs = level_pairs(tree, k, scheme)[drop_coarse:]
        self.spaces = [Space(m, d, dirichlet=dirichlet, coef=coef, coef_fine=tree, geometry=geometry)
                       for m, d in self.pairs]
        self.levels = []
        for l, S in enumerate(self.spaces):
            A = assemble_stiffness(S)
            P = prolongation(S, self.spaces[l - 1]) if l > 0 else None
            self.levels.append(solvers.Level(A, P, cheb_degree))
        for L in self.levels[1:]:
            L.setup_smoother()
        self.coarse = solvers.CoarseDirect(self.levels[0].A)

    @property
    def fine(self):
        return self.levels[-1]

    def vcycle(self, b):
        return solvers.vcycle(self.levels, b, self.coarse)

    def fmg(self, b, cycles=1):
        return solvers.fmg(self.levels, b, self.coarse, cycles)

    def solve(self, b, rtol=1e-10, max_it=200, flexible=False):
        return solvers.pcg(self.fine.A, b, self.vcycle, rtol, max_it, flexible)
