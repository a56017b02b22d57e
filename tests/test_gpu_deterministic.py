"""Deterministic mode (mfmg_level_desc.deterministic): the operator adds its
cells' contributions in cell order, the restriction, diagonal and load
vector run colour by colour with plain adds.  Every operation, repeated in
one context and in a second context set up the same way, gives bitwise
identical results, and the results still match the FP64 oracle (operator,
diagonal, load, transfers, V-cycle, solve); the default mode (atomics) is
compared with it to the usual tolerances."""
import functools

import numpy as np
import pytest
import torch

import synth
from oracle import solvers
from oracle.hierarchy import Hierarchy
from oracle.space import assemble_load, constant

from helpers import DESCS, SCHEME_CODES, oracle_tree, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
CASES = [("cfg1", 2, "h", None), ("small", 4, "h_then_p", None), ("spheres_small", 3, "hp", None),
         ("small", 2, "h", "bump")]


@functools.lru_cache(maxsize=None)
def solvers_for(name, k, scheme, geom):
    from paper_2203_12292_amd import mfmg
    print(f"[setup] deterministic {name} k={k} {scheme} geometry={geom}", flush=True)
    g = synth.GEOM_BUMP8 if geom == "bump" else None
    mk = lambda det: mfmg.Solver(mfmg.Mesh(DESCS[name]), k, SCHEME_CODES[scheme], geometry=g, max_rhs=3,
                                 deterministic=det)
    H = Hierarchy(oracle_tree(name), k, scheme, geometry=g)
    A, B, D = mk(True), mk(True), mk(False)
    P = [perm_from_codes(V.codes_array(), A.dof_codes(l)) for l, V in enumerate(H.spaces)]
    return H, A, B, D, P


def put(x, perm):
    g = np.zeros(len(perm))
    g[perm] = x
    return torch.tensor(g, dtype=torch.float64, device=DEV)


def get(t, perm):
    return t.double().cpu().numpy()[perm]


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name,k,scheme,geom", CASES)
def test_bitwise_repeatable_and_oracle(name, k, scheme, geom):
    H, A, B, D, P = solvers_for(name, k, scheme, geom)
    rng = np.random.default_rng(11)
    for l, L in enumerate(H.levels):
        n = L.A.shape[0]
        for nv in (1, 3):
            x = rng.uniform(-1, 1, (n, nv))
            xs = torch.zeros((n, nv), dtype=torch.float64, device=DEV)
            for v in range(nv):
                xs[:, v] = put(x[:, v], P[l])
            xs = xs.contiguous().view(-1)
            outs = []
            for S in (A, A, B):
                y = torch.empty_like(xs)
                S.vmult(l, y, xs, n_vec=nv)
                outs.append(y)
            torch.cuda.synchronize()
            assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2]), (l, nv)
            yd = torch.empty_like(xs)
            D.vmult(l, yd, xs, n_vec=nv)
            for v in range(nv):
                ref = L.A @ x[:, v]
                assert rel(get(outs[0].view(n, nv)[:, v], P[l]), ref) < 1e-12, (l, v)
                assert rel(get(yd.view(n, nv)[:, v], P[l]), ref) < 1e-12, (l, v)
        d = [torch.empty(n, dtype=torch.float64, device=DEV) for _ in range(3)]
        A.diagonal(l, d[0])
        A.diagonal(l, d[1])
        B.diagonal(l, d[2])
        torch.cuda.synchronize()
        assert torch.equal(d[0], d[1]) and torch.equal(d[0], d[2]), l
        assert rel(get(d[0], P[l]), L.A.diagonal()) < 1e-12, l
        if l > 0:
            nc = H.levels[l - 1].A.shape[0]
            xc = rng.uniform(-1, 1, nc)
            xf = rng.uniform(-1, 1, n)
            r = [torch.zeros(nc, dtype=torch.float64, device=DEV) for _ in range(3)]
            p = [torch.zeros(n, dtype=torch.float64, device=DEV) for _ in range(3)]
            for i, S in enumerate((A, A, B)):
                S.restrict_add(l, r[i], put(xf, P[l]))
                S.prolongate_add(l, p[i], put(xc, P[l - 1]))
            torch.cuda.synchronize()
            assert torch.equal(r[0], r[1]) and torch.equal(r[0], r[2]), l
            assert torch.equal(p[0], p[1]) and torch.equal(p[0], p[2]), l
            assert rel(get(r[0], P[l - 1]), L.P.T @ xf) < 1e-12, l
            assert rel(get(p[0], P[l]), L.P @ xc) < 1e-12, l
    # load vector, V-cycle and solve
    nf = H.fine.A.shape[0]
    bs = [torch.zeros(nf, dtype=torch.float64, device=DEV) for _ in range(3)]
    for i, S in enumerate((A, A, B)):
        S.rhs(bs[i])
    torch.cuda.synchronize()
    assert torch.equal(bs[0], bs[1]) and torch.equal(bs[0], bs[2])
    bo = assemble_load(H.spaces[-1], constant(1.0))
    assert rel(get(bs[0], P[-1]), bo) < 1e-12
    for l in range(1, A.n_levels):
        H.levels[l].lmin, H.levels[l].lmax = A.smoother_range(l)
        assert A.smoother_range(l) == B.smoother_range(l), l
    b = rng.uniform(-1, 1, nf)
    xs = []
    for S in (A, A, B):
        xv = torch.zeros(nf, dtype=torch.float64, device=DEV)
        S.vcycle(xv, put(b, P[-1]))
        xs.append(xv)
    torch.cuda.synchronize()
    assert torch.equal(xs[0], xs[1]) and torch.equal(xs[0], xs[2])
    assert rel(get(xs[0], P[-1]), H.vcycle(b)) < 1e-11
    sol, its = [], []
    for S in (A, A, B):
        xv = torch.zeros(nf, dtype=torch.float64, device=DEV)
        st = S.solve(xv, bs[0], rtol=1e-12, max_it=100)
        sol.append(xv)
        its.append(st["iterations"])
    torch.cuda.synchronize()
    assert torch.equal(sol[0], sol[1]) and torch.equal(sol[0], sol[2]), its
    xo = solvers.direct_solve(H.fine.A, bo)
    err = np.linalg.norm(get(sol[0], P[-1]) - xo) / np.linalg.norm(xo)
    print(f"[deterministic] {name} k={k} {scheme} {geom}: {its[0]} iterations, error {err:.2e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("name,k", [("small", 4), ("cfg1", 2)])
def test_local_smoothing_bitwise_repeatable(name, k):
    """Local smoothing in the deterministic mode: the solve (copies to and
    from the levels, edge-truncated smoothers, transfers, load vector) gives
    the same bits twice in one context and in a second one."""
    from paper_2203_12292_amd import mfmg
    mk = lambda: mfmg.Solver(mfmg.Mesh(DESCS[name]), k, mfmg.SCHEME_LS, deterministic=True)
    A, B = mk(), mk()
    sols = []
    for S in (A, A, B):
        b = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
        S.rhs(b)
        x = torch.zeros_like(b)
        st = S.solve(x, b, rtol=1e-10, max_it=100)
        assert st["converged"]
        sols.append(x)
    torch.cuda.synchronize()
    assert torch.equal(sols[0], sols[1]) and torch.equal(sols[0], sols[2])
