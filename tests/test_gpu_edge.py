"""Degenerate and edge cases on the GPU, checked against the oracle or against
properties that the FE space fixes exactly.

* A single Q1 cell with Dirichlet boundary has no free DoF: every call is a
  valid no-op on empty vectors and the solve converges at once.
* A single Q2 cell has one DoF; a uniform mesh has no hanging nodes.
* A zero right-hand side gives x = 0 without iterations.
* Without Dirichlet conditions (pure Neumann), the constants are the null
  space of the constrained operator, A 1 = 0, and u^T A u = |a|^2 vol(Omega)
  for every linear u = a.x (Q_k interpolates it exactly and the hanging-node
  constraints reproduce it); both pin the constraint handling independently
  of the oracle.  The singular problem is rejected by the solver calls.
"""
import functools

import numpy as np
import pytest
import torch

import synth
from oracle import octree, solvers
from oracle.space import Space, assemble_load, assemble_stiffness, constant

from helpers import DESCS, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None

EDGE = {
    "one_cell": synth.mesh_desc("one_cell", 1, 0.0, 1.0, 0, []),
    "uniform": synth.mesh_desc("uniform3_g1", 3, 0.0, 1.0, 1, []),
}


@functools.lru_cache(maxsize=None)
def solver(name, k, dirichlet=True):
    from paper_2203_12292_amd import mfmg
    desc = EDGE.get(name) or DESCS[name]
    print(f"[setup] mesh={name} k={k} dirichlet={dirichlet}", flush=True)
    return mfmg.Solver(mfmg.Mesh(desc), k, mfmg.SCHEME_H, dirichlet=dirichlet)


def oracle_space(name, k, dirichlet=True):
    desc = EDGE.get(name) or DESCS[name]
    return Space(octree.build_mesh(desc), k, dirichlet=dirichlet)


def zeros(n, nv=1):
    return torch.zeros((n, nv) if nv > 1 else n, dtype=torch.float64, device=DEV)


def test_single_q1_cell_has_no_dofs():
    S = solver("one_cell", 1)
    assert S.n_levels == 1 and S.n_dofs() == 0
    x, y = zeros(0), zeros(0)
    S.vmult(0, y, x)
    S.rhs(y)
    st = S.solve(x, y, rtol=1e-10, max_it=10)
    torch.cuda.synchronize()
    assert st["converged"] and st["iterations"] == 0


def test_single_q2_cell():
    S = solver("one_cell", 2)
    sp = oracle_space("one_cell", 2)
    A = assemble_stiffness(sp).toarray()
    assert S.n_dofs() == 1 and A.shape == (1, 1)
    x = torch.ones(1, dtype=torch.float64, device=DEV)
    y = torch.empty_like(x)
    S.vmult(0, y, x)
    b = zeros(1)
    S.rhs(b)
    xs = zeros(1)
    st = S.solve(xs, b, rtol=1e-12, max_it=10)
    torch.cuda.synchronize()
    assert abs(float(y[0]) - A[0, 0]) <= 1e-13 * abs(A[0, 0])
    b_ref = assemble_load(sp, constant(1.0))
    assert abs(float(b[0]) - b_ref[0]) <= 1e-13 * abs(b_ref[0])
    assert st["converged"] and abs(float(xs[0]) - b_ref[0] / A[0, 0]) <= 1e-12 * abs(b_ref[0] / A[0, 0])


@pytest.mark.parametrize("k", [1, 3])
def test_uniform_mesh_without_hanging_nodes(k):
    S = solver("uniform", k)
    sp = oracle_space("uniform", k)
    A = assemble_stiffness(sp)
    perm = perm_from_codes(sp.codes_array(), S.dof_codes(S.n_levels - 1))
    xo = np.random.default_rng(k).uniform(-1, 1, A.shape[0])
    xg = np.zeros(len(perm))
    xg[perm] = xo
    x = torch.tensor(xg, device=DEV)
    y = torch.empty_like(x)
    S.vmult(S.n_levels - 1, y, x)
    b = torch.zeros_like(x)
    S.rhs(b)
    xs = torch.zeros_like(x)
    st = S.solve(xs, b, rtol=1e-12, max_it=50)
    torch.cuda.synchronize()
    ref = A @ xo
    assert np.abs(y.cpu().numpy()[perm] - ref).max() <= 1e-12 * np.abs(ref).max()
    u = solvers.direct_solve(A, assemble_load(sp, constant(1.0)))
    assert st["converged"] and np.abs(xs.cpu().numpy()[perm] - u).max() <= 1e-10 * np.abs(u).max()


def test_zero_rhs_gives_zero_without_iterations():
    S = solver("small", 2)
    b = zeros(S.n_dofs())
    x = torch.full_like(b, 3.0)
    st = S.solve(x, b, rtol=1e-10, max_it=10)
    torch.cuda.synchronize()
    assert st["converged"] and st["iterations"] == 0 and float(x.abs().max()) == 0.0


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_neumann_constants_are_the_null_space(k):
    S = solver("small", k, dirichlet=False)
    for l in range(S.n_levels):
        n = S.n_dofs(l)
        one = torch.ones(n, dtype=torch.float64, device=DEV)
        y = torch.empty_like(one)
        d = torch.empty_like(one)
        S.vmult(l, y, one)
        S.diagonal(l, d)
        torch.cuda.synchronize()
        assert float(y.abs().max()) <= 1e-12 * float(d.abs().max()), (k, l)
        assert float(d.min()) > 0.0


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_neumann_linear_functions_have_exact_energy(k):
    """u = a.x at the DoF positions: u^T A u = |a|^2 on the unit cube."""
    S = solver("small", k, dirichlet=False)
    sp = oracle_space("small", k, dirichlet=False)
    perm = perm_from_codes(sp.codes_array(), S.dof_codes(S.n_levels - 1))
    a = np.array([0.3, -1.1, 0.7])
    ug = np.zeros(len(perm))
    ug[perm] = sp.dof_points() @ a
    u = torch.tensor(ug, device=DEV)
    y = torch.empty_like(u)
    S.vmult(S.n_levels - 1, y, u)
    torch.cuda.synchronize()
    energy = float(torch.dot(u, y))
    assert abs(energy - float(a @ a)) <= 1e-11 * float(a @ a)


def test_neumann_problem_rejects_the_solver_calls():
    from paper_2203_12292_amd import mfmg
    S = solver("small", 2, dirichlet=False)
    b = torch.ones(S.n_dofs(), dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    for call in (lambda: S.solve(x, b), lambda: S.vcycle(x, b), lambda: S.coarse_solve(zeros(S.n_dofs(0)),
                                                                                    zeros(S.n_dofs(0)))):
        with pytest.raises(mfmg.MfmgError) as e:
            call()
        assert e.value.code == mfmg.ERR_UNSUPPORTED
