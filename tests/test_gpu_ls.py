"""GPU parity of geometric local smoothing (Section 2.1; Algorithms 1-2,
local-smoothing branch) against the FP64 oracle, DoFs matched by their exact
position codes.

Level calls on every local-smoothing level (operator with edge rows,
diagonal, refinement-edge flags, smoothing on A_SS, transfers), the copy to
and from the levels, one V-cycle, and the PCG solve.  Tolerances as in the
global-coarsening tests: 1e-12 (FP64) relative to the largest entry, 1e-11
for a V-cycle and 1e-10 for solutions.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import solvers
from oracle.local_smoothing import LSHierarchy
from oracle.space import assemble_load, constant

from helpers import DESCS, oracle_hierarchy, oracle_tree, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
CASES = [("tiny", 1), ("tiny", 2), ("small_m1", 3), ("small", 4)]


@functools.lru_cache(maxsize=None)
def oracle_ls(name, k):
    return LSHierarchy(oracle_tree(name), k)


@functools.lru_cache(maxsize=None)
def gpu_ls(name, k, dtypes=(), coarse_p=False):
    from paper_2203_12292_amd import mfmg
    print(f"[setup] local smoothing mesh={name} k={k} dtypes={dtypes} coarse_p={coarse_p}", flush=True)
    return mfmg.Solver(mfmg.Mesh(DESCS[name]), k, mfmg.SCHEME_LS_THEN_P if coarse_p else mfmg.SCHEME_LS,
                       level_dtypes=list(dtypes))


@functools.lru_cache(maxsize=None)
def perms(name, k):
    """Oracle-to-library DoF permutations: (per level, active mesh)."""
    H, S = oracle_ls(name, k), gpu_ls(name, k)
    lv = [perm_from_codes(V.codes_array(), S.dof_codes(l)) for l, V in enumerate(H.spaces)]
    return lv, perm_from_codes(H.active.codes_array(), S.dof_codes(-1))


def to_gpu(x, perm, dtype=torch.float64):
    g = np.zeros(len(perm))
    g[perm] = x
    return torch.tensor(g, dtype=dtype, device=DEV)


def from_gpu(t, perm):
    return t.double().cpu().numpy()[perm]


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name,k", CASES)
def test_levels_operator_diagonal_edge(name, k):
    H, S = oracle_ls(name, k), gpu_ls(name, k)
    P, _ = perms(name, k)
    assert S.n_levels == len(H.levels)
    rng = np.random.default_rng(k)
    for l, L in enumerate(H.levels):
        n_edge, flags = S.level_edge(l)
        assert n_edge == L.E.size and np.array_equal(flags[P[l]].astype(bool), L.space.edge)
        x = rng.uniform(-1, 1, L.n)
        y = torch.empty(L.n, dtype=torch.float64, device=DEV)
        S.vmult(l, y, to_gpu(x, P[l]))
        d = torch.empty_like(y)
        S.diagonal(l, d)
        torch.cuda.synchronize()
        print(f"[ls] {name} k={k} level {l}: {L.n} DoFs, {n_edge} on the edge", flush=True)
        assert rel_err(from_gpu(y, P[l]), L.A_full @ x) < 1e-12
        assert rel_err(from_gpu(d, P[l]), L.A_full.diagonal()) < 1e-12


@pytest.mark.parametrize("name,k", CASES)
def test_smoothing_acts_on_interior_dofs(name, k):
    """From x = 0 with b_E = 0: x_S is the Chebyshev smoother of A_SS, x_E = 0.
    From x with x_E != 0: the smoother solves A_SS x_S = b_S - A_SE x_E and
    keeps x_E (the edge step folded into the smoother's operator)."""
    H, S = oracle_ls(name, k), gpu_ls(name, k)
    P, _ = perms(name, k)
    rng = np.random.default_rng(5)
    for l in range(1, len(H.levels)):
        L = H.levels[l]
        sm = L.smoother
        lmin, lmax = S.smoother_range(l)
        assert abs(lmax - sm.lmax) <= 1e-10 * sm.lmax and abs(lmin - sm.lmin) <= 1e-10 * sm.lmin
        b = np.zeros(L.n)
        b[L.S] = rng.uniform(-1, 1, L.S.size)
        x = torch.zeros(L.n, dtype=torch.float64, device=DEV)
        S.smooth(l, x, to_gpu(b, P[l]), x_is_zero=True)
        x0 = np.zeros(L.n)
        x0[L.E] = rng.uniform(-1, 1, L.E.size)
        x0[L.S] = rng.uniform(-1, 1, L.S.size)
        x2 = to_gpu(x0, P[l])
        S.smooth(l, x2, to_gpu(b, P[l]))
        torch.cuda.synchronize()
        ref = solvers.chebyshev(sm.A, sm.Dinv, b[L.S], None, sm.degree, lmin, lmax)
        xg = from_gpu(x, P[l])
        assert rel_err(xg[L.S], ref) < 1e-12 and np.abs(xg[L.E]).max(initial=0.0) == 0.0
        bS = b[L.S] - L.A_SE @ x0[L.E]
        ref2 = solvers.chebyshev(sm.A, sm.Dinv, bS, x0[L.S], sm.degree, lmin, lmax)
        xg2 = from_gpu(x2, P[l])
        assert rel_err(xg2[L.S], ref2) < 1e-12 and np.array_equal(xg2[L.E], x0[L.E])


@pytest.mark.parametrize("name,k", CASES)
def test_transfers_between_levels(name, k):
    H, S = oracle_ls(name, k), gpu_ls(name, k)
    P, _ = perms(name, k)
    rng = np.random.default_rng(9)
    for l in range(1, len(H.levels)):
        Pm = H.levels[l].P
        xc = rng.uniform(-1, 1, Pm.shape[1])
        xf = rng.uniform(-1, 1, Pm.shape[0])
        yf = torch.zeros(Pm.shape[0], dtype=torch.float64, device=DEV)
        yc = torch.zeros(Pm.shape[1], dtype=torch.float64, device=DEV)
        S.prolongate_add(l, yf, to_gpu(xc, P[l - 1]))
        S.restrict_add(l, yc, to_gpu(xf, P[l]))
        torch.cuda.synchronize()
        assert rel_err(from_gpu(yf, P[l]), Pm @ xc) < 1e-12
        assert rel_err(from_gpu(yc, P[l - 1]), Pm.T @ xf) < 1e-12


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small_m1", 3)])
def test_copy_to_and_from_levels(name, k):
    H, S = oracle_ls(name, k), gpu_ls(name, k)
    P, PA = perms(name, k)
    b = np.random.default_rng(4).uniform(-1, 1, H.A.shape[0])
    bg = to_gpu(b, PA)
    ref = H.copy_to_mg(b)
    back = torch.full_like(bg, np.nan)
    for l, L in enumerate(H.levels):
        bl = torch.full((L.n,), 7.0, dtype=torch.float64, device=DEV)
        S.copy_to_mg(l, bl, bg)
        S.copy_from_mg(l, back, bl)
        torch.cuda.synchronize()
        assert np.array_equal(from_gpu(bl, P[l]), ref[l]), l
    assert np.array_equal(from_gpu(back, PA), b)


@pytest.mark.parametrize("name,k", CASES)
def test_vcycle(name, k):
    H, S = oracle_ls(name, k), gpu_ls(name, k)
    _, PA = perms(name, k)
    for l in range(1, S.n_levels):  # identical smoother intervals on both sides
        H.levels[l].smoother.lmin, H.levels[l].smoother.lmax = S.smoother_range(l)
    b = np.random.default_rng(2).uniform(-1, 1, H.A.shape[0])
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    S.vcycle(xg, to_gpu(b, PA))
    torch.cuda.synchronize()
    assert rel_err(from_gpu(xg, PA), H.vcycle(b)) < 1e-11


@pytest.mark.parametrize("name,k", [("tiny", 2), ("cfg1", 2), ("small", 4)])
def test_solve_fp64(name, k):
    """PCG with the local-smoothing V-cycle reaches the direct solution in as
    many iterations as the oracle's, at least as many as global coarsening."""
    S = gpu_ls(name, k)
    _, PA = perms(name, k) if name != "cfg1" else (None, None)
    H = oracle_ls(name, k) if name != "cfg1" else None
    G = oracle_hierarchy(name, k)
    bg = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    S.rhs(bg)
    xg = torch.zeros_like(bg)
    st = S.solve(xg, bg, rtol=1e-12, max_it=80)
    torch.cuda.synchronize()
    b_o = assemble_load(G.spaces[-1], constant(1.0))
    xo = solvers.direct_solve(G.fine.A, b_o)
    pa = PA if PA is not None else perm_from_codes(G.spaces[-1].codes_array(), S.dof_codes(-1))
    err = np.linalg.norm(from_gpu(xg, pa) - xo) / np.linalg.norm(xo)
    _, it_gc, _ = G.solve(b_o, rtol=1e-12)
    print(f"[ls solve] {name} k={k}: {st['iterations']} it (GC {it_gc}), err {err:.2e}", flush=True)
    assert st["converged"] and err < 1e-10 and st["iterations"] >= it_gc
    if H is not None:
        _, it_o, _ = H.solve(b_o, rtol=1e-12)
        assert abs(st["iterations"] - it_o) <= 1


def test_solve_fp32_levels():
    """FP32 local-smoothing V-cycle inside FP64 CG reaches 1e-10."""
    G = oracle_hierarchy("cfg1", 2)
    S = gpu_ls("cfg1", 2, (1,))
    bg = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    S.rhs(bg)
    xg = torch.zeros_like(bg)
    st = S.solve(xg, bg, rtol=1e-10, max_it=60)
    torch.cuda.synchronize()
    pa = perm_from_codes(G.spaces[-1].codes_array(), S.dof_codes(-1))
    xo = solvers.direct_solve(G.fine.A, assemble_load(G.spaces[-1], constant(1.0)))
    err = np.linalg.norm(from_gpu(xg, pa) - xo) / np.linalg.norm(xo)
    print(f"[ls solve fp32] {st['iterations']} it, err {err:.2e}", flush=True)
    assert st["converged"] and err < 1e-8


def test_active_level_has_no_smoother():
    from paper_2203_12292_amd import mfmg
    S = gpu_ls("tiny", 2)
    x = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    with pytest.raises(mfmg.MfmgError) as e:
        S.smooth(mfmg.LEVEL_ACTIVE, x, x.clone())
    assert e.value.code == mfmg.ERR_UNSUPPORTED


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small", 4)])
def test_vcycle_with_polynomial_coarse_levels(name, k):
    """Local smoothing down to the coarse grid, then polynomial levels there
    (degrees 1, 2, ..., floor(k/2)): V-cycle parity and the FP64 solve."""
    H = LSHierarchy(oracle_tree(name), k, coarse_p=True)
    S = gpu_ls(name, k, coarse_p=True)
    assert S.n_levels == len(H.levels)
    for l in range(S.n_levels):
        assert S.level_info(l)["degree"] == H.levels[l].space.k
    for l in range(1, S.n_levels):
        H.levels[l].smoother.lmin, H.levels[l].smoother.lmax = S.smoother_range(l)
    PA = perm_from_codes(H.active.codes_array(), S.dof_codes(-1))
    b = np.random.default_rng(2).uniform(-1, 1, H.A.shape[0])
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    S.vcycle(xg, to_gpu(b, PA))
    bg = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    S.rhs(bg)
    xs = torch.zeros_like(bg)
    st = S.solve(xs, bg, rtol=1e-12, max_it=80)
    torch.cuda.synchronize()
    assert rel_err(from_gpu(xg, PA), H.vcycle(b)) < 1e-11
    b_o = assemble_load(H.active, constant(1.0))
    xo = solvers.direct_solve(H.A, b_o)
    err = np.linalg.norm(from_gpu(xs, PA) - xo) / np.linalg.norm(xo)
    print(f"[ls+p solve] {name} k={k}: {st['iterations']} it, err {err:.2e}", flush=True)
    assert st["converged"] and err < 1e-10


def test_fmg_is_not_offered_under_local_smoothing():
    from paper_2203_12292_amd import mfmg
    S = gpu_ls("tiny", 2)
    x = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    with pytest.raises(mfmg.MfmgError) as e:
        S.fmg(x, x.clone())
    assert e.value.code == mfmg.ERR_UNSUPPORTED
