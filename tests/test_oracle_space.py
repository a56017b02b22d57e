"""Oracle space, constraints, assembly and transfer pinned to mathematics.

* A = A^T, SPD with Dirichlet constraints; without Dirichlet constraints
  A 1 = 0 and u^T A u = |a|^2 vol for u = a.x (exact for Gauss (k+1)^3).
* Continuity across hanging faces: the discrete function takes the same value
  on both sides at random points of every hanging face.
* Uniform Q1 meshes give the textbook 27-point stencil.
* Galerkin identity P^T A_f P = A_c for nested spaces (global coarsening and
  polynomial coarsening): ties constraints, transfer and level operators.
* P reproduces coarse interpolants of polynomials.
* Discretisation error O(h^{k+1}) for -Lap u = 3 pi^2 u, u = sin sin sin.
"""
import numpy as np
import pytest

import synth
from oracle import fe, octree, solvers
from oracle.space import (Space, assemble_load, assemble_stiffness, coefficient, distribute_values,
                          l2_error, prolongation)


@pytest.fixture(scope="module")
def tiny():
    return octree.build_mesh(synth.CFG1_TINY)


@pytest.fixture(scope="module")
def small():
    return octree.build_mesh(synth.small_mesh())


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_symmetric_positive_definite(small, k):
    S = Space(small, k)
    A = assemble_stiffness(S).toarray()
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A)[0] > 0


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_neumann_kernel_and_linear_energy(tiny, k):
    S = Space(tiny, k, dirichlet=False)
    A = assemble_stiffness(S)
    assert np.abs(A @ np.ones(S.n_dofs)).max() < 1e-13
    pts = S.dof_points()
    a = np.array([0.3, -1.2, 0.7])
    u = pts @ a + 0.25
    assert abs(u @ (A @ u) - a @ a) < 1e-12


def _hanging_faces(space):
    """(fine cell, face axis, side) of faces whose neighbour is a coarser leaf."""
    out = []
    for cell in space.cells:
        l, i, j, m = cell
        if l == 0:
            continue
        ext = space.tree.n0 << l
        for ax in range(3):
            for side in (0, 1):
                q = [i, j, m]
                q[ax] += 1 if side else -1
                if not (0 <= q[ax] < ext):
                    continue
                nb = space.index.find_leaf(l, *q)
                if nb is not None and nb[0] == l - 1:
                    out.append((cell, ax, side))
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_continuity_across_hanging_faces(small, k):
    S = Space(small, k)
    x = np.random.default_rng(k).standard_normal(S.n_dofs)
    faces = _hanging_faces(S)
    assert faces
    rng = np.random.default_rng(1)
    for cell, ax, side in faces:
        l, i, j, m = cell
        h = S.tree.h(l)
        lo = S.tree.lo + h * np.array([i, j, m], float)
        for _ in range(3):
            p = lo + h * rng.uniform(0, 1, 3)
            p[ax] = lo[ax] + (h if side else 0.0)
            q = [i, j, m]
            q[ax] += 1 if side else -1
            other = S.index.find_leaf(l, *q)
            vals = []
            for c in (cell, other):
                hc = S.tree.h(c[0])
                loc = (p - (S.tree.lo + hc * np.array(c[1:], float))) / hc
                vals.append(fe.basis_at(k, loc[None])[0] @ distribute_values(S, c, x))
            assert abs(vals[0] - vals[1]) < 1e-12 * (1 + abs(vals[0]))


def test_uniform_q1_stencil():
    t = octree.Octree(4)
    S = Space(t, 1)
    A = assemble_stiffness(S).toarray()
    h = 0.25
    pts = S.dof_points()
    centre = np.argmin(np.abs(pts - 0.5).sum(axis=1))
    for j in range(S.n_dofs):
        d = np.round(np.abs(pts[j] - pts[centre]) / h).astype(int)
        if d.max() > 1:
            assert A[centre, j] == 0
            continue
        nz = int((d > 0).sum())
        want = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[nz] * h
        assert abs(A[centre, j] - want) < 1e-15


@pytest.mark.parametrize("k,scheme", [(1, "h"), (2, "h"), (3, "h"), (4, "p"), (2, "hp"), (4, "hp")])
def test_galerkin_identity(tiny, k, scheme):
    if scheme == "h":
        coarse_tree = tiny.coarsened()
        Sf, Sc = Space(tiny, k), Space(coarse_tree, k)
    elif scheme == "hp":  # mesh coarsened and degree halved in one step
        Sf, Sc = Space(tiny, k), Space(tiny.coarsened(), k // 2)
    else:
        Sf, Sc = Space(tiny, k), Space(tiny, k // 2)
    P = prolongation(Sf, Sc)
    Af, Ac = assemble_stiffness(Sf), assemble_stiffness(Sc)
    G = (P.T @ Af @ P - Ac).toarray()
    assert np.abs(G).max() < 1e-13 * abs(Ac).max()


@pytest.mark.parametrize("kf,kc,h", [(2, 2, True), (4, 2, False), (3, 1, False), (6, 3, False), (4, 2, True),
                                     (6, 3, True), (2, 1, True)])
def test_prolongation_reproduces_polynomials(small, kf, kc, h):
    coarse_tree = small.coarsened() if h else small
    Sf, Sc = Space(small, kf, dirichlet=False), Space(coarse_tree, kc, dirichlet=False)
    P = prolongation(Sf, Sc)

    def u(p):
        return 0.3 + p[:, 0] * (1 - 2 * p[:, 1]) + (p[:, 2] ** kc if kc > 1 else p[:, 2])
    assert np.abs(P @ u(Sc.dof_points()) - u(Sf.dof_points())).max() < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2])
def test_convergence_rate(k):
    def u(p):
        return np.sin(np.pi * p[:, 0]) * np.sin(np.pi * p[:, 1]) * np.sin(np.pi * p[:, 2])

    def f(p):
        return 3 * np.pi ** 2 * u(p)
    errs = []
    for n0 in (2, 4, 8):
        t = octree.Octree(n0)
        # locally refined towards a corner, so hanging nodes are present
        t.refine_where(synth.BALL, (0.0, 0.0, 0.0, 0.45))
        S = Space(t, k)
        A = assemble_stiffness(S)
        x = solvers.direct_solve(A, assemble_load(S, f))
        errs.append(l2_error(S, x, u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 1 - 0.25, (errs, rates)


def test_bfloat16_rounding():
    """Cell coefficients are rounded to bfloat16: 8 significant bits, ties to even."""
    from oracle.space import bf16_round
    assert bf16_round(1.0 / 3.0) == 0.333984375          # 0x3EAB
    assert bf16_round(1000.0) == 1000.0 and bf16_round(0.5) == 0.5
    assert bf16_round(1.0 + 2.0 ** -8) == 1.0            # halfway, to the even neighbour
    assert bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7


@pytest.mark.parametrize("k", [1, 2, 4])
def test_cellwise_coefficient_energy_of_linear_functions(small, k):
    """-div(c grad u) with c constant per cell, without Dirichlet conditions:
    constants span the null space, and u = a.x (exact in Q_k, also across
    hanging faces) has energy |a|^2 sum_e c_e h_e^3 (exact with Gauss
    quadrature); c = 4 everywhere gives exactly 4 times the Laplacian."""
    coef = synth.coef_desc(synth.COEF_BALL, (0.2, 0.3, 0.1, 0.45, 1000.0, 1.0 / 3.0))
    S = Space(small, k, dirichlet=False, coef=coef)
    A = assemble_stiffness(S)
    assert np.abs(A @ np.ones(S.n_dofs)).max() < 1e-10 * abs(A).max()
    a = np.array([0.3, -1.1, 0.7])
    u = S.dof_points() @ a
    vol = sum(S.cell_coef(c) * S.cell_h(c) ** 3 for c in S.cells)
    values = {S.cell_coef(c) for c in S.cells}
    assert values == {1000.0, 0.333984375}
    assert abs(u @ (A @ u) - (a @ a) * vol) < 1e-11 * (a @ a) * vol
    S4 = Space(small, k, coef=synth.coef_desc(synth.COEF_CONST, (4.0,)))
    S1 = Space(small, k)
    assert np.abs((assemble_stiffness(S4) - 4.0 * assemble_stiffness(S1)).toarray()).max() == 0.0


def test_coarse_cell_coefficient_is_the_leaf_average():
    """A coarser level's cell coefficient (before rounding) is the volume
    average over the finest leaves it covers: summed over any coarse mesh of
    the hierarchy, c_K |K| reproduces the fine integral of the coefficient."""
    from oracle.space import CellCoefficient
    fine = octree.build_mesh(synth.small_mesh())
    cc = CellCoefficient(synth.COEF_INCLUSION, fine)
    c = coefficient(synth.COEF_INCLUSION)
    total = sum(c(fine.lo + fine.h(l) * (ijk + 0.5)) * fine.h(l) ** 3
                for l, cells in fine.all_leaves() for ijk in cells.astype(float))
    for mesh in octree.gc_sequence(fine)[1:]:
        coarse = sum(cc.raw((l, *map(int, ijk))) * mesh.h(l) ** 3 for l, cells in mesh.all_leaves() for ijk in cells)
        assert abs(coarse - total) <= 1e-12 * total
