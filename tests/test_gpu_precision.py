"""Per-operation error of the FP32 and bfloat16 level arithmetic against the
FP64 oracle (the mixed-precision extension: FP32 levels, bfloat16 storage
with FP32 arithmetic on the coarsest ones).  Every hot-path level call runs
on levels stored in that type, and its result is compared with the oracle's
FP64 result for the same (rounded) inputs, relative to the largest entry.
The measured errors are printed per result; the bounds are those of the
operator tests: FP32 2e-5, bfloat16 2e-2 (8 significant bits; the Chebyshev
smoother stores x and d in the level type after each of its 3 steps, 3e-2).
The transfers add into a vector of the level type: a DoF receives one
addition per transfer group it belongs to (at most 8) and each rounds to the
storage type, so their bound is (1 + 8) u (max|base| + max|P x|) / max|P x|
with the unit roundoff u of the type (2^-8 for bfloat16), or the FP32
operator bound if larger.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import solvers

from helpers import DESCS, oracle_hierarchy, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
CODE = {torch.float32: 1, torch.bfloat16: 2}
TOL = {torch.float32: 2e-5, torch.bfloat16: 2e-2}


@functools.lru_cache(maxsize=None)
def solver(name, k, dtype):
    from paper_2203_12292_amd import mfmg
    print(f"[setup] {name} k={k} all levels {dtype}", flush=True)
    return mfmg.Solver(mfmg.Mesh(DESCS[name]), k, mfmg.SCHEME_H, level_dtypes=[CODE[dtype]])


@functools.lru_cache(maxsize=None)
def perms(name, k, dtype):
    H = oracle_hierarchy(name, k)
    S = solver(name, k, dtype)
    return [perm_from_codes(H.spaces[l].codes_array(), S.dof_codes(l)) for l in range(S.n_levels)]


def put(x, perm, dtype):
    g = np.zeros(len(perm))
    g[perm] = x
    return torch.tensor(g, dtype=dtype, device=DEV)


def get(t, perm):
    return t.double().cpu().numpy()[perm]


def err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small", 4)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_level_ops_against_fp64_oracle(name, k, dtype):
    H = oracle_hierarchy(name, k)
    S = solver(name, k, dtype)
    P = perms(name, k, dtype)
    rng = np.random.default_rng(17)
    tol = TOL[dtype]
    worst = {}
    u = {torch.float32: 2.0 ** -24, torch.bfloat16: 2.0 ** -8}[dtype]

    def add_bound(base, ref):
        return max(tol, 9 * u * (np.abs(base).max() + np.abs(ref).max()) / np.abs(ref).max())

    def report(op, l, e, bound):
        print(f"[{dtype} err] {name} Q{k} level {l} {op}: {e:.2e} (bound {bound:.0e})", flush=True)
        worst[op] = max(worst.get(op, 0.0), e)
        assert e < bound, (op, l, e)

    for l in range(S.n_levels):
        A = H.levels[l].A
        n = A.shape[0]
        xg = put(rng.uniform(-1, 1, n), P[l], dtype)
        x = get(xg, P[l])  # the rounded input the GPU sees
        yg = torch.empty_like(xg)
        S.vmult(l, yg, xg)
        torch.cuda.synchronize()
        report("vmult", l, err(get(yg, P[l]), A @ x), tol)
        bg = put(rng.uniform(-1, 1, n), P[l], dtype)
        b = get(bg, P[l])
        rg = torch.empty_like(xg)
        S.residual(l, rg, bg, xg)
        torch.cuda.synchronize()
        report("residual", l, err(get(rg, P[l]), b - A @ x), tol)
        if l == 0:
            cg = torch.empty_like(bg)
            S.coarse_solve(cg, bg)
            torch.cuda.synchronize()
            report("coarse solve", l, err(get(cg, P[l]), solvers.direct_solve(A, b)), tol)
            continue
        L = H.levels[l]
        lam = S.smoother_range(l)
        sg = torch.zeros_like(bg)
        S.smooth(l, sg, bg, x_is_zero=True)
        torch.cuda.synchronize()
        report("smooth (x0 = 0)", l, err(get(sg, P[l]), solvers.chebyshev(L.A, L.Dinv, b, None, 3, *lam)),
               1.5 * tol)
        sg = xg.clone()
        S.smooth(l, sg, bg, x_is_zero=False)
        torch.cuda.synchronize()
        report("smooth", l, err(get(sg, P[l]), solvers.chebyshev(L.A, L.Dinv, b, x, 3, *lam)), 1.5 * tol)
        Pm = L.P
        base = put(rng.uniform(-1, 1, n), P[l], dtype)
        base_used = get(base, P[l])
        xc = put(rng.uniform(-1, 1, Pm.shape[1]), P[l - 1], dtype)
        S.prolongate_add(l, base, xc)
        torch.cuda.synchronize()
        ref = Pm @ get(xc, P[l - 1])
        report("prolongate_add", l, err(get(base, P[l]) - base_used, ref), add_bound(base_used, ref))
        basec = put(rng.uniform(-1, 1, Pm.shape[1]), P[l - 1], dtype)
        basec_used = get(basec, P[l - 1])
        S.restrict_add(l, basec, xg)
        torch.cuda.synchronize()
        ref = Pm.T @ x
        report("restrict_add", l, err(get(basec, P[l - 1]) - basec_used, ref), add_bound(basec_used, ref))
    print(f"[{dtype} worst] {name} Q{k}: " + ", ".join(f"{op} {e:.1e}" for op, e in worst.items()), flush=True)
