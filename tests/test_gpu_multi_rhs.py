"""Several vectors in one call (DoF-major interleaved layout [n][n_vec]):
every hot-path call against the FP64 oracle applied column by column, on the
sphere-cut mesh family of the p-multigrid workload (Q6 -> Q3 -> Q1, then
global coarsening), as in the benchmark's eight-right-hand-side solve.

Tolerances as for one vector: FP64 1e-12 and FP32 2e-5 relative to the
largest entry of each column.
"""
import functools

import numpy as np
import pytest
import torch

import synth
from oracle import solvers
from oracle.space import assemble_load, gaussian_sum

from helpers import DESCS, SCHEME_CODES, oracle_hierarchy, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
TOL = {torch.float64: 1e-12, torch.float32: 2e-5}
NAME, K, SCHEME, NV = "spheres_small", 6, "p_then_h", 8


@functools.lru_cache(maxsize=None)
def solver(dtypes=()):
    from paper_2203_12292_amd import mfmg
    print(f"[setup] mesh={NAME} k={K} scheme={SCHEME} dtypes={dtypes} max_rhs={NV}", flush=True)
    return mfmg.Solver(mfmg.Mesh(DESCS[NAME]), K, SCHEME_CODES[SCHEME], level_dtypes=list(dtypes), max_rhs=NV)


@functools.lru_cache(maxsize=None)
def perms():
    H = oracle_hierarchy(NAME, K, SCHEME)
    S = solver()
    return [perm_from_codes(H.spaces[l].codes_array(), S.dof_codes(l)) for l in range(S.n_levels)]


def to_gpu(X, perm, dtype=torch.float64):
    G = np.zeros((len(perm), X.shape[1]))
    G[perm] = X
    return torch.tensor(G, dtype=dtype, device=DEV).contiguous()


def from_gpu(t, perm):
    return t.double().cpu().numpy()[perm]


def col_err(A, B):
    """Largest over columns of max|a - b| / max|b|."""
    return max(np.abs(A[:, c] - B[:, c]).max() / max(np.abs(B[:, c]).max(), 1e-300) for c in range(B.shape[1]))


@pytest.mark.parametrize("nv", [3, NV])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_vmult_multi(nv, dtype):
    H = oracle_hierarchy(NAME, K, SCHEME)
    S, P = solver(), perms()
    rng = np.random.default_rng(11)
    for l in range(S.n_levels):
        A = H.levels[l].A
        X = rng.uniform(-1, 1, (A.shape[0], nv))
        xg = to_gpu(X, P[l], dtype)
        yg = torch.empty_like(xg)
        S.vmult(l, yg, xg, n_vec=nv)
        torch.cuda.synchronize()
        assert col_err(from_gpu(yg, P[l]), A @ from_gpu(xg, P[l])) < TOL[dtype], (l, nv)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_transfer_multi(dtype):
    H = oracle_hierarchy(NAME, K, SCHEME)
    S, P = solver(), perms()
    rng = np.random.default_rng(12)
    for l in range(1, S.n_levels):
        Pm = H.levels[l].P
        Xc = rng.uniform(-1, 1, (Pm.shape[1], NV))
        base = rng.uniform(-1, 1, (Pm.shape[0], NV))
        dst = to_gpu(base, P[l], dtype)
        base_r = from_gpu(dst, P[l])
        xc = to_gpu(Xc, P[l - 1], dtype)
        S.prolongate_add(l, dst, xc, n_vec=NV)
        torch.cuda.synchronize()
        assert col_err(from_gpu(dst, P[l]) - base_r, Pm @ from_gpu(xc, P[l - 1])) < 10 * TOL[dtype], l
        Rf = rng.uniform(-1, 1, (Pm.shape[0], NV))
        basec = rng.uniform(-1, 1, (Pm.shape[1], NV))
        dstc = to_gpu(basec, P[l - 1], dtype)
        basec_r = from_gpu(dstc, P[l - 1])
        rf = to_gpu(Rf, P[l], dtype)
        S.restrict_add(l, dstc, rf, n_vec=NV)
        torch.cuda.synchronize()
        assert col_err(from_gpu(dstc, P[l - 1]) - basec_r, Pm.T @ from_gpu(rf, P[l])) < 10 * TOL[dtype], l


def test_smooth_and_residual_multi():
    H = oracle_hierarchy(NAME, K, SCHEME)
    S, P = solver(), perms()
    rng = np.random.default_rng(13)
    lam = (0.09, 1.8)
    for l in range(1, S.n_levels):
        L = H.levels[l]
        B = rng.uniform(-1, 1, (L.A.shape[0], NV))
        X0 = rng.uniform(-1, 1, (L.A.shape[0], NV))
        bg = to_gpu(B, P[l])
        xg = torch.zeros_like(bg)
        S.smooth(l, xg, bg, x_is_zero=True, lam=lam, n_vec=NV)
        ref = np.stack([solvers.chebyshev(L.A, L.Dinv, B[:, c], None, 3, *lam) for c in range(NV)], axis=1)
        torch.cuda.synchronize()
        assert col_err(from_gpu(xg, P[l]), ref) < 1e-12, ("smooth x0=0", l)
        xg = to_gpu(X0, P[l])
        S.smooth(l, xg, bg, x_is_zero=False, lam=lam, n_vec=NV)
        ref = np.stack([solvers.chebyshev(L.A, L.Dinv, B[:, c], X0[:, c], 3, *lam) for c in range(NV)], axis=1)
        torch.cuda.synchronize()
        assert col_err(from_gpu(xg, P[l]), ref) < 1e-12, ("smooth", l)
        rg = torch.empty_like(bg)
        S.residual(l, rg, bg, to_gpu(X0, P[l]), n_vec=NV)
        torch.cuda.synchronize()
        assert col_err(from_gpu(rg, P[l]), B - L.A @ X0) < 1e-12, ("residual", l)


def test_vcycle_multi():
    H = oracle_hierarchy(NAME, K, SCHEME)
    S, P = solver(), perms()
    for l in range(1, S.n_levels):
        H.levels[l].lmin, H.levels[l].lmax = S.smoother_range(l)
    B = np.random.default_rng(14).uniform(-1, 1, (H.fine.A.shape[0], NV))
    xg = torch.zeros((len(P[-1]), NV), dtype=torch.float64, device=DEV)
    S.vcycle(xg, to_gpu(B, P[-1]), n_vec=NV)
    torch.cuda.synchronize()
    ref = np.stack([H.vcycle(B[:, c]) for c in range(NV)], axis=1)
    assert col_err(from_gpu(xg, P[-1]), ref) < 1e-11


@functools.lru_cache(maxsize=None)
def reference_solutions():
    """Eight Gaussian loads (four terms each) and their exact solutions (one
    sparse factorisation for all eight columns)."""
    H = oracle_hierarchy(NAME, K, SCHEME)
    params = np.stack(synth.gaussian_rhs_batch(NV))
    B = np.stack([assemble_load(H.spaces[-1], gaussian_sum(params[c])) for c in range(NV)], axis=1)
    print("[oracle] direct solve of the eight loads", flush=True)
    return params, B, solvers.direct_solve(H.fine.A, B)


@pytest.mark.parametrize("dtypes", [(), (1,)])
def test_rhs_and_solve_multi(dtypes):
    """Eight Gaussian right-hand sides assembled in one call and solved in
    lock step; FP64 levels, or FP32 levels inside FP64 CG."""
    from paper_2203_12292_amd import mfmg
    H = oracle_hierarchy(NAME, K, SCHEME)
    S, P = solver(dtypes), perms()
    params, B, Xo = reference_solutions()
    n = len(P[-1])
    bg = torch.zeros((n, NV), dtype=torch.float64, device=DEV)
    S.rhs(bg, mfmg.RHS_GAUSS, params, n_terms=params.shape[1], n_vec=NV)
    assert col_err(from_gpu(bg, P[-1]), B) < 1e-12
    xg = torch.zeros_like(bg)
    st = S.solve(xg, bg, rtol=1e-12, max_it=100, flexible=bool(dtypes), n_vec=NV)
    torch.cuda.synchronize()
    X = from_gpu(xg, P[-1])
    for c in range(NV):
        res = np.linalg.norm(B[:, c] - H.fine.A @ X[:, c]) / np.linalg.norm(B[:, c])
        err = np.linalg.norm(X[:, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c])
        print(f"[solve {dtypes}] rhs {c}: {st['iterations']} it, residual {res:.2e}, err {err:.2e}")
        assert res < 1.01e-12 and err < 1e-9, c
    assert st["converged"] and 3 <= st["iterations"] <= 40


def test_fmg_multi():
    """Full multigrid on eight interleaved right-hand sides against the oracle."""
    H = oracle_hierarchy(NAME, K, SCHEME)
    S, P = solver(), perms()
    for l in range(1, S.n_levels):
        H.levels[l].lmin, H.levels[l].lmax = S.smoother_range(l)
    B = np.random.default_rng(15).uniform(-1, 1, (H.fine.A.shape[0], NV))
    xg = torch.zeros((len(P[-1]), NV), dtype=torch.float64, device=DEV)
    S.fmg(xg, to_gpu(B, P[-1]), cycles=1, n_vec=NV)
    torch.cuda.synchronize()
    ref = np.stack([H.fmg(B[:, c]) for c in range(NV)], axis=1)
    assert col_err(from_gpu(xg, P[-1]), ref) < 1e-11


@pytest.mark.parametrize("scheme", ["ls", "hp"])
def test_vcycle_multi_other_schemes(scheme):
    """Local smoothing and the one-step h+p hierarchy with four interleaved
    right-hand sides: each column equals the oracle's V-cycle."""
    from oracle.hierarchy import Hierarchy
    from oracle.local_smoothing import LSHierarchy
    from paper_2203_12292_amd import mfmg
    from helpers import oracle_tree
    nv, name, k = 4, "small", 4
    print(f"[setup] mesh={name} k={k} scheme={scheme} max_rhs={nv}", flush=True)
    if scheme == "ls":
        H = LSHierarchy(oracle_tree(name), k)
        S = mfmg.Solver(mfmg.Mesh(DESCS[name]), k, mfmg.SCHEME_LS, max_rhs=nv)
        smoothers = [L.smoother for L in H.levels]
        active = H.active
    else:
        H = Hierarchy(oracle_tree(name), k, "hp")
        S = mfmg.Solver(mfmg.Mesh(DESCS[name]), k, mfmg.SCHEME_HP, max_rhs=nv)
        smoothers = H.levels
        active = H.spaces[-1]
    for l in range(1, S.n_levels):
        smoothers[l].lmin, smoothers[l].lmax = S.smoother_range(l)
    PA = perm_from_codes(active.codes_array(), S.dof_codes(-1))
    B = np.random.default_rng(16).uniform(-1, 1, (len(PA), nv))
    xg = torch.zeros((len(PA), nv), dtype=torch.float64, device=DEV)
    S.vcycle(xg, to_gpu(B, PA), n_vec=nv)
    torch.cuda.synchronize()
    ref = np.stack([H.vcycle(B[:, c]) for c in range(nv)], axis=1)
    assert col_err(from_gpu(xg, PA), ref) < 1e-11
    S.close()
