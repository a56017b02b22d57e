"""The oracle's mapped cells (oracle.geometry) pinned to facts that do not
depend on its quadrature code:

* no motion: the quadrature assembly equals the closed form c h A_ref;
* affine maps (parallelepipeds): the integrands are polynomials that Gauss
  quadrature integrates exactly and the levels are nested, so the Galerkin
  identity P^T A_f P = A_c holds to rounding on a mesh with hanging nodes;
* trilinear maps: a function linear in the physical coordinates, u = a.x,
  is in every Q_k space of such a mesh (the map is Q1), its gradient is a
  everywhere and |det J| has degree <= 2 per variable, so u^T A u equals
  |a|^2 vol exactly; the interior bump keeps the boundary, vol = 1;
  constants are in the kernel without Dirichlet conditions;
* trilinear maps: the L2 error of the discrete solution of -Lap u = f for a
  smooth u on the deformed mesh falls like h^(k+1) (a wrong Jacobian
  transform stalls it).
"""
import numpy as np
import pytest

import synth
from oracle import geometry, octree, solvers
from oracle.hierarchy import Hierarchy
from oracle.space import Space, assemble_load, assemble_stiffness, l2_error, prolongation

BUMP = {"kind": 2, "params": [0.08, 1.0, -0.7, 0.5]}
SHEAR = {"kind": 1, "params": [1.3, 0.4, -0.2, 0.9, 0.3, 1.1]}


@pytest.fixture(scope="module")
def small():
    return octree.build_mesh(synth.small_mesh())


def test_no_motion_equals_closed_form(small):
    for k in (1, 2, 3):
        A0 = assemble_stiffness(Space(small, k)).toarray()
        A1 = assemble_stiffness(Space(small, k, geometry={"kind": 2, "params": [0.0, 1.0, 1.0, 1.0]})).toarray()
        assert np.abs(A0 - A1).max() < 1e-13 * np.abs(A0).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_affine_galerkin_identity(small, k):
    Sf = Space(small, k, geometry=SHEAR)
    Sc = Space(small.coarsened(), k, geometry=SHEAR)
    P = prolongation(Sf, Sc)
    Af, Ac = assemble_stiffness(Sf), assemble_stiffness(Sc)
    G = (P.T @ Af @ P - Ac).toarray()
    assert np.abs(G).max() < 1e-13 * abs(Ac).max()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_trilinear_linear_energy_and_kernel(small, k):
    S = Space(small, k, dirichlet=False, geometry=BUMP)
    A = assemble_stiffness(S)
    x = S.physical_dof_points()
    # the interior bump moves interior vertices but not the boundary
    assert np.abs(x - S.dof_points()).max() > 1e-3
    a = np.array([0.7, -1.1, 0.4])
    u = x @ a
    assert abs(u @ (A @ u) - a @ a) < 1e-12
    assert np.abs(A @ np.ones(S.n_dofs)).max() < 1e-12
    assert np.abs((A - A.T).toarray()).max() < 1e-13


def test_trilinear_dirichlet_operator_is_spd(small):
    A = assemble_stiffness(Space(small, 2, geometry=BUMP)).toarray()
    assert np.linalg.eigvalsh(A)[0] > 0


def test_map_vertices_and_jacobian():
    """Vertices of a fine cell are moved coarse-cell points; the Jacobian is
    the finite-difference derivative of the map."""
    t = octree.Octree(2)
    g = geometry.CoarseTrilinearGeometry(t, BUMP)
    cell = (2, 5, 2, 6)  # level 2: in coarse cell (1, 0, 1)
    X = g.coarse_vertices(1, 0, 1)
    # the cell's corner (0,0,0) is the coarse point t = (1/4, 2/4, 2/4)
    tt = np.array([0.25, 0.5, 0.5])
    w = [(1 - tt[0]) if a == 0 else tt[0] for a in (0, 1)]
    N = np.array([((1 - tt[0]) if v & 1 == 0 else tt[0]) * ((1 - tt[1]) if v & 2 == 0 else tt[1]) *
                  ((1 - tt[2]) if v & 4 == 0 else tt[2]) for v in range(8)])
    assert np.allclose(g.points(cell, np.zeros((1, 3)))[0], N @ X, atol=1e-15)
    xi = np.array([[0.3, 0.6, 0.2]])
    J = g.jacobians(cell, xi)[0]
    h = 1e-6
    for e in range(3):
        d = np.zeros((1, 3))
        d[0, e] = h
        fd = (g.points(cell, xi + d) - g.points(cell, xi - d))[0] / (2 * h)
        assert np.allclose(J[:, e], fd, atol=1e-9)


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2])
def test_trilinear_convergence_rate(k):
    def u(p):
        return np.sin(np.pi * p[:, 0]) * np.sin(np.pi * p[:, 1]) * np.sin(np.pi * p[:, 2])

    def f(p):
        return 3 * np.pi ** 2 * u(p)
    errs = []
    for n0 in (2, 4, 8):
        t = octree.Octree(n0)
        t.refine_where(synth.BALL, (0.0, 0.0, 0.0, 0.45))
        S = Space(t, k, geometry=BUMP)
        A = assemble_stiffness(S)
        x = solvers.direct_solve(A, assemble_load(S, f))
        errs.append(l2_error(S, x, u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 1 - 0.3, (errs, rates)


def test_hierarchy_passes_the_geometry(small):
    H = Hierarchy(small, 2, geometry=SHEAR)
    assert all(S.geometry is not None for S in H.spaces)
