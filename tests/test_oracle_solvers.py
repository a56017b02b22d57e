"""Oracle smoother, V-cycle and PCG pinned to closed forms and invariants.

* Chebyshev (Section 3.3): on a generalised eigenvector v (A v = lam D v) with
  b = 0, degree-m smoothing maps v to p_m(lam) v with the scaled Chebyshev
  residual polynomial p_m(lam) = T_m((theta - lam)/delta) / T_m(theta/delta).
* The Lanczos estimate never exceeds the largest eigenvalue of D^{-1}A.
* The V-cycle of Algorithm 2 (pre- and post-smoothing by the same Chebyshev
  polynomial, exact coarse solve) is a symmetric operator and a contraction
  in the energy norm.
* PCG converges to the direct solution.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import octree, solvers
from oracle.hierarchy import Hierarchy
from oracle.space import Space, assemble_load, assemble_stiffness, constant


@pytest.fixture(scope="module")
def hier():
    return Hierarchy(octree.build_mesh(synth.CFG1_TINY), 2, "h")


def _cheb_T(m, x):
    return np.cosh(m * np.arccosh(x)) if abs(x) >= 1 else np.cos(m * np.arccos(x))


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_chebyshev_on_eigenvectors(m):
    t = octree.build_mesh(synth.small_mesh())
    A = assemble_stiffness(Space(t, 2)).toarray()
    D = np.diag(A)
    lam, V = sla.eigh(A, np.diag(D))
    lmin, lmax = 0.25 * lam[-1] / 4, 1.1 * lam[-1]
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    for idx in (0, len(lam) // 3, len(lam) - 1):
        v = V[:, idx]
        out = solvers.chebyshev(A, 1.0 / D, np.zeros_like(v), v, m, lmin, lmax)
        p = _cheb_T(m, (theta - lam[idx]) / delta) / _cheb_T(m, theta / delta)
        assert np.abs(out - p * v).max() < 1e-12 * np.abs(v).max()


def test_chebyshev_zero_start_matches_general(hier):
    L = hier.levels[-1]
    b = np.random.default_rng(0).standard_normal(L.A.shape[0])
    x1 = solvers.chebyshev(L.A, L.Dinv, b, None, 3, L.lmin, L.lmax)
    x2 = solvers.chebyshev(L.A, L.Dinv, b, np.zeros_like(b), 3, L.lmin, L.lmax)
    assert np.abs(x1 - x2).max() < 1e-14 * np.abs(x1).max()


def test_lambda_estimate_below_max(hier):
    for L in hier.levels[1:]:
        lam = solvers.estimate_lambda_max(L.A, L.Dinv)
        D = L.A.diagonal()
        true = sla.eigh(L.A.toarray(), np.diag(D), eigvals_only=True)[-1]
        assert lam <= true * (1 + 1e-12)
        assert lam > 0.8 * true


def test_vcycle_symmetric_and_contracting(hier):
    n = hier.fine.A.shape[0]
    rng = np.random.default_rng(3)
    v, w = rng.standard_normal(n), rng.standard_normal(n)
    Bv, Bw = hier.vcycle(v), hier.vcycle(w)
    assert abs(w @ Bv - v @ Bw) < 1e-12 * abs(w @ Bv)
    # energy-norm contraction of I - B A on random vectors
    A = hier.fine.A
    for _ in range(3):
        e = rng.standard_normal(n)
        e2 = e - hier.vcycle(A @ e)
        assert np.sqrt(e2 @ (A @ e2)) < 0.5 * np.sqrt(e @ (A @ e))


def test_pcg_matches_direct(hier):
    b = assemble_load(hier.spaces[-1], constant(1.0))
    x, it, hist = hier.solve(b, 1e-12)
    xd = solvers.direct_solve(hier.fine.A, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert 4 <= it <= 15
    assert hist[-1] <= 1e-12


def test_flexible_cg_same_as_standard_for_fixed_preconditioner(hier):
    b = assemble_load(hier.spaces[-1], constant(1.0))
    x1, it1, _ = hier.solve(b, 1e-10)
    x2, it2, _ = hier.solve(b, 1e-10, flexible=True)
    assert it1 == it2
    assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x1)


@pytest.mark.parametrize("drop", [1, 2])
def test_early_coarse_switch(drop):
    """The direct coarse solve on a finer level (with hanging nodes) still gives
    a symmetric positive definite V-cycle, and PCG reaches the direct solution
    in no more iterations than with the full hierarchy."""
    from helpers import oracle_hierarchy, oracle_tree
    tree = oracle_tree("cfg1")
    H = Hierarchy(tree, 2, "h", drop_coarse=drop)
    full = oracle_hierarchy("cfg1", 2)
    assert len(H.levels) == len(full.levels) - drop
    assert any(H.spaces[0].cell_has_hanging(c) for c in H.spaces[0].cells)
    rng = np.random.default_rng(21)
    u, v = rng.standard_normal(H.fine.A.shape[0]), rng.standard_normal(H.fine.A.shape[0])
    Bu, Bv = H.vcycle(u), H.vcycle(v)
    assert abs(u @ Bv - v @ Bu) <= 1e-12 * abs(u @ Bv) and u @ Bu > 0
    b = assemble_load(H.spaces[-1], constant(1.0))
    x, it, _ = H.solve(b, rtol=1e-10)
    _, it_full, _ = full.solve(b, rtol=1e-10)
    xd = solvers.direct_solve(H.fine.A, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd) and it <= it_full


def test_switch_on_finest_level_is_exact():
    """Leaving out every level but the finest makes the V-cycle the exact
    inverse: PCG converges in one iteration."""
    from helpers import oracle_tree
    tree = oracle_tree("tiny")
    n = len(Hierarchy(tree, 2, "h").levels)
    H = Hierarchy(tree, 2, "h", drop_coarse=n - 1)
    b = assemble_load(H.spaces[-1], constant(1.0))
    _, it, _ = H.solve(b, rtol=1e-12)
    assert len(H.levels) == 1 and it == 1


def _sine_problem(g, k):
    from oracle.space import l2_error
    desc = synth.mesh_desc(f"cube2_g{g}_ball", 2, 0.0, 1.0, g, [(synth.BALL, (0.0, 0.0, 0.0, 0.45))])
    H = Hierarchy(octree.build_mesh(desc), k, "h")

    def u(p):
        return np.sin(np.pi * p[:, 0]) * np.sin(np.pi * p[:, 1]) * np.sin(np.pi * p[:, 2])
    b = assemble_load(H.spaces[-1], lambda p: 3 * np.pi ** 2 * u(p))
    return H, b, u, l2_error


@pytest.mark.parametrize("k,gs", [(1, (1, 2, 3)), (2, (1, 2))])
def test_fmg_reaches_discretisation_accuracy(k, gs):
    """FMG with two V-cycles per level solves to the size of the
    discretisation error at every mesh size (the defining property of full
    multigrid): its algebraic error in the energy norm stays below a quarter
    of the discretisation error ||u - u_h||_A (from Galerkin orthogonality,
    ||u - u_h||_A^2 = ||u||_A^2 - u_h^T A u_h with ||u||_A^2 = 3 pi^2 / 8 for
    u = sin(pi x) sin(pi y) sin(pi z)), and its L2 error stays within 1.2x
    of u_h's and converges at the rate h^(k+1)."""
    e_fmg = []
    for g in gs:
        H, b, u, l2_error = _sine_problem(g, k)
        S = H.spaces[-1]
        xh = solvers.direct_solve(H.fine.A, b)
        x = H.fmg(b, cycles=2)
        e_disc = np.sqrt(3 * np.pi ** 2 / 8 - xh @ (H.fine.A @ xh))
        e_alg = np.sqrt((x - xh) @ (H.fine.A @ (x - xh)))
        assert e_alg <= 0.25 * e_disc, (g, e_alg, e_disc)
        e_fmg.append(l2_error(S, x, u))
        assert e_fmg[-1] <= 1.2 * l2_error(S, xh, u), g
    rates = np.log2(np.array(e_fmg[:-1]) / np.array(e_fmg[1:]))
    assert rates[-1] > k + 1 - 0.5, rates


def test_fmg_with_many_cycles_is_the_discrete_solution():
    H, b, _, _ = _sine_problem(1, 2)
    x = H.fmg(b, cycles=30)
    xd = solvers.direct_solve(H.fine.A, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
