"""V-cycles of the outer solver replayed from HIP graphs (`graph_vcycle`):
every solve, repeated with the program's own eager work and synchronisations
between them, matches the eager solver (same kernels in the same order: same
iteration count, results equal up to the last-bit differences that the
order of the operator's LDS atomics can cause, which two eager solves show as
well), for the standard and the flexible CG (two alternating vector pairs),
FP64 and mixed-precision levels, global coarsening and local smoothing; the
switched-off coarse correction keeps the eager path.
"""
import numpy as np
import pytest
import torch

import synth
from helpers import DESCS

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


@pytest.mark.parametrize("scheme,dtypes,flexible", [("h", (), False), ("h", (2, 2, 1), True), ("ls", (), False)])
def test_graph_solves_equal_eager_solves(scheme, dtypes, flexible):
    from paper_2203_12292_amd import mfmg
    sc = mfmg.SCHEME_LS if scheme == "ls" else mfmg.SCHEME_H
    mesh = mfmg.Mesh(DESCS["cfg1"])
    print(f"[setup] cfg1 k=2 scheme={scheme} dtypes={dtypes} flexible={flexible}", flush=True)
    E = mfmg.Solver(mesh, 2, sc, level_dtypes=list(dtypes))
    G = mfmg.Solver(mesh, 2, sc, level_dtypes=list(dtypes), graph_vcycle=True)
    n = E.n_dofs()
    rng = np.random.default_rng(5)
    for rep in range(3):
        params = synth.gaussian_rhs_training(rep)
        b = torch.zeros(n, dtype=torch.float64, device=DEV)
        E.rhs(b, mfmg.RHS_GAUSS, params, n_terms=params.shape[0])
        xe, xg = torch.zeros_like(b), torch.zeros_like(b)
        se = E.solve(xe, b, rtol=1e-10, max_it=60, flexible=flexible)
        xe2 = torch.zeros_like(b)
        E.solve(xe2, b, rtol=1e-10, max_it=60, flexible=flexible)
        # eager work of the program itself between the replays
        y = torch.empty_like(b)
        G.vmult(G.n_levels - 1 if scheme != "ls" else mfmg.LEVEL_ACTIVE, y,
                torch.tensor(rng.uniform(-1, 1, n), device=DEV))
        torch.cuda.synchronize()
        sg = G.solve(xg, b, rtol=1e-10, max_it=60, flexible=flexible)
        torch.cuda.synchronize()
        scale = float(xe.abs().max())
        d_graph = float((xg - xe).abs().max()) / scale
        d_eager = float((xe2 - xe).abs().max()) / scale
        print(f"[graph] rep {rep}: {se['iterations']} / {sg['iterations']} it, graph vs eager {d_graph:.1e}, "
              f"eager vs eager {d_eager:.1e}", flush=True)
        assert se["converged"] and sg["iterations"] == se["iterations"]
        assert d_graph <= 1e-12, rep
    E.close()
    G.close()


def test_other_coarse_modes_stay_eager():
    """With the coarse correction switched off (the comparison mode of the
    learned correction) the graph option changes nothing."""
    from paper_2203_12292_amd import mfmg
    mesh = mfmg.Mesh(DESCS["cfg1"])
    E = mfmg.Solver(mesh, 2, mfmg.SCHEME_H)
    G = mfmg.Solver(mesh, 2, mfmg.SCHEME_H, graph_vcycle=True)
    b = torch.zeros(E.n_dofs(), dtype=torch.float64, device=DEV)
    E.rhs(b)
    out = []
    for S in (E, G):
        S.net_mode(mfmg.COARSE_ZERO, 0.5)
        x = torch.zeros_like(b)
        st = S.solve(x, b, rtol=1e-10, max_it=100, flexible=True)
        torch.cuda.synchronize()
        out.append((x, st))
    assert out[0][1]["converged"] and out[1][1]["iterations"] == out[0][1]["iterations"]
    assert float((out[0][0] - out[1][0]).abs().max()) <= 1e-12 * float(out[0][0].abs().max())
    E.close()
    G.close()


def test_graph_solves_with_changing_vector_count():
    """One context with max_rhs = 8: a solve of one vector, then of 8
    interleaved vectors that reuse the same work buffers, then one vector
    again.  Each (x, b, n_vec) gets its own eager first cycle and its own
    graph, and every graph solve equals the eager solve."""
    from paper_2203_12292_amd import mfmg
    mesh = mfmg.Mesh(DESCS["cfg1"])
    print("[setup] cfg1 k=2 max_rhs=8 graph and eager", flush=True)
    E = mfmg.Solver(mesh, 2, mfmg.SCHEME_H, max_rhs=8)
    G = mfmg.Solver(mesh, 2, mfmg.SCHEME_H, max_rhs=8, graph_vcycle=True)
    n = E.n_dofs()
    for nv in (1, 8, 1, 8):
        params = np.concatenate([synth.gaussian_rhs(500 + v, 2, 0.05, 0.3, "normal", 0.0, 1.0)
                                 for v in range(nv)])
        b = torch.zeros(n * nv, dtype=torch.float64, device=DEV)
        E.rhs(b, mfmg.RHS_GAUSS, params, n_terms=2, n_vec=nv)
        out = []
        for S in (E, G):
            for _ in range(2):  # the second solve of G replays its graphs
                x = torch.zeros_like(b)
                st = S.solve(x, b, rtol=1e-10, max_it=60, n_vec=nv)
                torch.cuda.synchronize()
            out.append((x, st))
        scale = float(out[0][0].abs().max())
        d = float((out[1][0] - out[0][0]).abs().max()) / scale
        print(f"[graph nv={nv}] {out[0][1]['iterations']} / {out[1][1]['iterations']} it, graph vs eager {d:.1e}",
              flush=True)
        assert out[0][1]["converged"] and out[1][1]["iterations"] == out[0][1]["iterations"]
        assert d <= 1e-12
    E.close()
    G.close()
