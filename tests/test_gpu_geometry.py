"""Mapped cells (an affine shear: parallelepipeds; an interior bump: general
trilinear cells) against the FP64 oracle, which integrates every element
matrix and load by textbook Gauss quadrature with the Jacobian at each point
(oracle/geometry.py).  Element by element after matching DoFs by position
code, on meshes with hanging nodes: the operator of every level (FP64 1e-12,
FP32 2e-5 of the largest entry), its diagonal (1e-12), the load vector
(1e-12), the transfers (unchanged by the geometry: the levels are nested),
the V-cycle and the solve against the oracle's direct solution (1e-10)."""
import functools

import numpy as np
import pytest
import torch

import synth
from oracle import solvers
from oracle.hierarchy import Hierarchy
from oracle.space import assemble_load, constant, gaussian_sum

from helpers import DESCS, oracle_tree, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
GEOMS = {"shear": synth.GEOM_SHEAR, "bump": synth.GEOM_BUMP8}


@functools.lru_cache(maxsize=None)
def pair(name, k, geom):
    from paper_2203_12292_amd import mfmg
    print(f"[setup] {name} k={k} geometry={geom}", flush=True)
    H = Hierarchy(oracle_tree(name), k, geometry=GEOMS[geom])
    S = mfmg.Solver(mfmg.Mesh(DESCS[name]), k, geometry=GEOMS[geom])
    P = [perm_from_codes(H.spaces[l].codes_array(), S.dof_codes(l)) for l in range(S.n_levels)]
    return H, S, P


def put(x, perm, dtype=torch.float64):
    g = np.zeros(len(perm))
    g[perm] = x
    return torch.tensor(g, dtype=dtype, device=DEV)


def get(t, perm):
    return t.double().cpu().numpy()[perm]


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


CASES = [("tiny", 1, "bump"), ("tiny", 2, "shear"), ("tiny", 2, "bump"), ("small", 3, "bump"),
         ("small", 4, "shear"), ("small", 4, "bump")]


@pytest.mark.parametrize("name,k,geom", CASES)
def test_mapped_operator_diagonal_and_load(name, k, geom):
    from paper_2203_12292_amd import mfmg
    H, S, P = pair(name, k, geom)
    rng = np.random.default_rng(k)
    for l in range(S.n_levels):
        A = H.levels[l].A
        x = rng.uniform(-1, 1, A.shape[0])
        for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
            xg = put(x, P[l], dtype)
            yg = torch.empty_like(xg)
            S.vmult(l, yg, xg)
            torch.cuda.synchronize()
            e = rel(get(yg, P[l]), A @ get(xg, P[l]))
            print(f"[geometry {geom}] {name} Q{k} level {l} vmult {dtype}: {e:.1e}", flush=True)
            assert e < tol, (l, dtype, e)
        d = torch.empty(A.shape[0], dtype=torch.float64, device=DEV)
        S.diagonal(l, d)
        torch.cuda.synchronize()
        assert rel(get(d, P[l]), A.diagonal()) < 1e-12, l
    b = torch.empty(S.n_dofs(), dtype=torch.float64, device=DEV)
    S.rhs(b)
    assert rel(get(b, P[-1]), assemble_load(H.spaces[-1], constant(1.0))) < 1e-12
    g = synth.gaussian_rhs(7, 3, 0.1, 0.3, "normal", DESCS[name]["lo"], DESCS[name]["hi"])
    S.rhs(b, mfmg.RHS_GAUSS, g, n_terms=3)
    assert rel(get(b, P[-1]), assemble_load(H.spaces[-1], gaussian_sum(g))) < 1e-12


@pytest.mark.parametrize("name,k,geom", [("tiny", 2, "bump"), ("small", 4, "bump"), ("small", 3, "shear")])
def test_mapped_vcycle_and_solve(name, k, geom):
    H, S, P = pair(name, k, geom)
    for l in range(1, S.n_levels):
        H.levels[l].lmin, H.levels[l].lmax = S.smoother_range(l)
    b = np.random.default_rng(2).uniform(-1, 1, H.fine.A.shape[0])
    xg = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    S.vcycle(xg, put(b, P[-1]))
    torch.cuda.synchronize()
    assert rel(get(xg, P[-1]), H.vcycle(b)) < 1e-11
    bg = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    S.rhs(bg)
    xs = torch.zeros_like(bg)
    st = S.solve(xs, bg, rtol=1e-12, max_it=80)
    torch.cuda.synchronize()
    xo = solvers.direct_solve(H.fine.A, assemble_load(H.spaces[-1], constant(1.0)))
    err = np.linalg.norm(get(xs, P[-1]) - xo) / np.linalg.norm(xo)
    print(f"[geometry {geom}] {name} Q{k} solve: {st['iterations']} it, err {err:.1e}", flush=True)
    assert st["converged"] and err < 1e-10


def test_mapped_smoother_interval_matches_oracle():
    H, S, P = pair("small", 4, "bump")
    for l in range(1, S.n_levels):
        lmin, lmax = S.smoother_range(l)
        assert abs(lmax - H.levels[l].lmax) < 1e-10 * H.levels[l].lmax


def test_geometry_refused_for_local_smoothing_and_inverted_maps():
    from paper_2203_12292_amd import mfmg
    mesh = mfmg.Mesh(DESCS["tiny"])
    with pytest.raises(mfmg.MfmgError) as e:
        mfmg.Solver(mesh, 2, mfmg.SCHEME_LS, geometry=synth.GEOM_BUMP8)
    assert e.value.code == mfmg.ERR_UNSUPPORTED
    with pytest.raises(mfmg.MfmgError) as e:
        mfmg.Solver(mesh, 2, geometry=synth.geom_desc(synth.GEOM_AFFINE, (1.0, 0.0, 0.0, 1.0, 0.0, -1.0)))
    assert e.value.code == mfmg.ERR_INVALID_ARG
