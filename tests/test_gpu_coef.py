"""GPU parity of the operator -div(c grad u) with a diffusion coefficient that
is constant per cell (c at a leaf's centre, the mean over the leaves a
coarser cell covers, rounded to bfloat16 as the cell mask carries it),
against the FP64 oracle: operator, diagonal and solves on every level
scheme, with high-contrast inclusions and a checkerboard.  Tolerances as for
the Laplacian.
"""
import functools

import numpy as np
import pytest
import torch

import synth
from oracle import solvers
from oracle.hierarchy import Hierarchy
from oracle.local_smoothing import LSHierarchy
from oracle.space import assemble_load, constant

from helpers import DESCS, SCHEME_CODES, oracle_tree, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
TOL = {torch.float64: 1e-12, torch.float32: 2e-5}
COEFS = {
    "inclusion": synth.COEF_INCLUSION,
    # an inclusion around a coarse cell centre of the 2^3 and 4^3 grids
    "corner_inclusion": synth.coef_desc(synth.COEF_BALL, (0.25, 0.25, 0.25, 0.3, 1000.0, 1.0)),
    "checker": synth.coef_desc(synth.COEF_CHECKER, (1.0, 0.01, 0.25, 0.0)),
}


@functools.lru_cache(maxsize=None)
def pair(name, k, scheme, coef):
    from paper_2203_12292_amd import mfmg
    print(f"[setup] mesh={name} k={k} scheme={scheme} coef={coef}", flush=True)
    if scheme == "ls":
        H = LSHierarchy(oracle_tree(name), k, coef=COEFS[coef])
        S = mfmg.Solver(mfmg.Mesh(DESCS[name]), k, mfmg.SCHEME_LS, coef=COEFS[coef])
        spaces = H.spaces
    else:
        H = Hierarchy(oracle_tree(name), k, scheme, coef=COEFS[coef])
        S = mfmg.Solver(mfmg.Mesh(DESCS[name]), k, SCHEME_CODES[scheme], coef=COEFS[coef])
        spaces = H.spaces
    P = [perm_from_codes(V.codes_array(), S.dof_codes(l)) for l, V in enumerate(spaces)]
    return H, S, P


def to_gpu(x, perm, dtype=torch.float64):
    g = np.zeros(len(perm))
    g[perm] = x
    return torch.tensor(g, dtype=dtype, device=DEV)


def from_gpu(t, perm):
    return t.double().cpu().numpy()[perm]


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name,k", [("tiny", 1), ("tiny", 2), ("small_m1", 3), ("small", 4), ("small", 5),
                                    ("small", 6)])
@pytest.mark.parametrize("coef", ["inclusion", "checker"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_operator_and_diagonal(name, k, coef, dtype):
    H, S, P = pair(name, k, "h", coef)
    rng = np.random.default_rng(k)
    for l, L in enumerate(H.levels):
        x = rng.uniform(-1, 1, L.A.shape[0])
        y = torch.empty(L.A.shape[0], dtype=dtype, device=DEV)
        S.vmult(l, y, to_gpu(x, P[l], dtype))
        d = torch.empty(L.A.shape[0], dtype=torch.float64, device=DEV)
        S.diagonal(l, d)
        torch.cuda.synchronize()
        xr = x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x
        assert rel_err(from_gpu(y, P[l]), L.A @ xr) < TOL[dtype], l
        assert rel_err(from_gpu(d, P[l]), L.A.diagonal()) < 1e-12, l


@pytest.mark.parametrize("name,k,scheme,coef", [("tiny", 2, "h", "corner_inclusion"),
                                                ("small", 4, "h_then_p", "inclusion"),
                                                ("small", 4, "ls", "corner_inclusion"), ("cfg1", 2, "h", "inclusion"),
                                                ("small", 4, "ls", "inclusion")])
def test_vcycle_and_solve(name, k, scheme, coef):
    H, S, P = pair(name, k, scheme, coef)
    levels = H.levels
    for l in range(1, S.n_levels):
        lo, hi = S.smoother_range(l)
        sm = levels[l].smoother if scheme == "ls" else levels[l]
        sm.lmin, sm.lmax = lo, hi
    PA = perm_from_codes((H.active if scheme == "ls" else H.spaces[-1]).codes_array(), S.dof_codes(-1))
    A = H.A if scheme == "ls" else H.fine.A
    b = np.random.default_rng(2).uniform(-1, 1, A.shape[0])
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    S.vcycle(xg, to_gpu(b, PA))
    bg = torch.zeros_like(xg)
    S.rhs(bg)
    xs = torch.zeros_like(xg)
    st = S.solve(xs, bg, rtol=1e-12, max_it=100)
    torch.cuda.synchronize()
    assert rel_err(from_gpu(xg, PA), H.vcycle(b)) < 1e-11
    space = H.active if scheme == "ls" else H.spaces[-1]
    xo = solvers.direct_solve(A, assemble_load(space, constant(1.0)))
    err = np.linalg.norm(from_gpu(xs, PA) - xo) / np.linalg.norm(xo)
    print(f"[solve] {name} k={k} {scheme} {coef}: {st['iterations']} it, err {err:.2e}", flush=True)
    assert st["converged"] and err < 1e-10


def fine_cell_values(S, space):
    """The coefficient of the finest level's cells in the library's cell
    order: the oracle's cell value (a leaf of the finest mesh takes c at its
    centre)."""
    lv, ijk = S.level_cells(S.n_levels - 1)
    vals = [space.coef.raw((int(l), int(i), int(j), int(m))) for l, (i, j, m) in zip(lv, ijk)]
    return torch.tensor(vals, dtype=torch.float64, device=DEV)


def check_against(H, S, P, tag):
    """Operator and diagonal of every level, the V-cycle (the library's
    Chebyshev intervals given to the oracle) and a solve against the FP64
    oracle of hierarchy H."""
    rng = np.random.default_rng(5)
    for l, L in enumerate(H.levels):
        x = rng.uniform(-1, 1, L.A.shape[0])
        y = torch.empty(L.A.shape[0], dtype=torch.float64, device=DEV)
        S.vmult(l, y, to_gpu(x, P[l]))
        d = torch.empty_like(y)
        S.diagonal(l, d)
        torch.cuda.synchronize()
        assert rel_err(from_gpu(y, P[l]), L.A @ x) < 1e-12, (tag, l)
        assert rel_err(from_gpu(d, P[l]), L.A.diagonal()) < 1e-12, (tag, l)
    for l in range(1, S.n_levels):
        H.levels[l].lmin, H.levels[l].lmax = S.smoother_range(l)
    b = rng.uniform(-1, 1, H.fine.A.shape[0])
    for rep in range(2):  # the second replays a captured cycle
        xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
        bg = to_gpu(b, P[-1])
        xs = torch.zeros_like(bg)
        st = S.solve(xs, bg, rtol=1e-12, max_it=100)
        torch.cuda.synchronize()
        xo = solvers.direct_solve(H.fine.A, b)
        err = np.linalg.norm(from_gpu(xs, P[-1]) - xo) / np.linalg.norm(xo)
        assert st["converged"] and err < 1e-10, (tag, rep, err)
    S.vcycle(xg, bg)
    torch.cuda.synchronize()
    assert rel_err(from_gpu(xg, P[-1]), H.vcycle(b)) < 1e-11, tag
    return st["iterations"]


@pytest.mark.parametrize("name,k,scheme", [("small", 2, "h"), ("small", 4, "h_then_p"), ("cfg1", 2, "h"),
                                           ("spheres_small", 3, "hp")])
def test_set_coefficient(name, k, scheme):
    """mfmg_set_coefficient on a solver set up with c = 1: the coefficient
    given on the finest cells reaches every level on the device, and every
    level's operator and diagonal, the V-cycle and a solve then match the FP64
    oracle set up with that coefficient; twice in a row (an inclusion, then a
    checkerboard), the solver replaying graph-captured V-cycles.  Values out
    of range are rejected and change nothing."""
    from paper_2203_12292_amd import mfmg
    print(f"[setup] set_coefficient mesh={name} k={k} scheme={scheme}", flush=True)
    S = mfmg.Solver(mfmg.Mesh(DESCS[name]), k, SCHEME_CODES[scheme], graph_vcycle=True)
    tree = oracle_tree(name)
    H0 = Hierarchy(tree, k, scheme)
    P = [perm_from_codes(V.codes_array(), S.dof_codes(l)) for l, V in enumerate(H0.spaces)]
    check_against(H0, S, P, "c = 1")
    for coef in ("inclusion", "checker"):
        H = Hierarchy(tree, k, scheme, coef=COEFS[coef])
        S.set_coefficient(fine_cell_values(S, H.spaces[-1]))
        its = check_against(H, S, P, coef)
        print(f"[set_coefficient] {name} k={k} {scheme} {coef}: {its} iterations", flush=True)
    bad = fine_cell_values(S, H.spaces[-1])
    bad[len(bad) // 2] = -1.0
    with pytest.raises(mfmg.MfmgError):
        S.set_coefficient(bad)
    check_against(H, S, P, "after a rejected update")


def test_set_coefficient_rejects_local_smoothing():
    from paper_2203_12292_amd import mfmg
    S = mfmg.Solver(mfmg.Mesh(DESCS["tiny"]), 2, mfmg.SCHEME_LS)
    n = S.level_info(S.n_levels - 1)["n_cells"]
    with pytest.raises(mfmg.MfmgError) as e:
        S.set_coefficient(torch.ones(n, dtype=torch.float64, device=DEV))
    assert e.value.code == mfmg.ERR_UNSUPPORTED
