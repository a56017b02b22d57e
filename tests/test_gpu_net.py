"""Learned coarse correction on the GPU.

* Gradients of the HIP forward/backward kernels (FP32) against the FP64
  oracle backward (itself checked by finite differences in
  test_oracle_mlp.py): relative error <= 1e-4.
* The exact coarse operator checks every prediction: a network that predicts 0
  is always rejected and the solve is then identical to the exact one.
* Gain: on a mesh whose coarse level matters (6^3 coarse cubes), after
  training on coarse right-hand sides recorded from the solver, the learned
  correction needs strictly fewer PCG iterations than no coarse correction;
  it is also compared with the exact coarse solve; all three reach a 1e-10
  relative residual in FP64 CG (flexible: the network makes the
  preconditioner non-linear) and the oracle's direct solution.  The
  network's output quality itself is not pinned ("parity unpinned").
"""
import functools

import numpy as np
import pytest
import torch

import synth
from oracle import mlp, solvers
from oracle.space import assemble_load, gaussian_sum

from helpers import DESCS, oracle_hierarchy, perm_from_codes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


@functools.lru_cache(maxsize=None)
def cfg1_solver():
    from paper_2203_12292_amd import mfmg
    print("[setup] cfg1 Q2 solver with learned correction", flush=True)
    return mfmg.Solver(mfmg.Mesh(synth.CFG1), 2)


def test_net_gradient_matches_oracle():
    S = cfg1_solver()
    n = S.net_n_params()
    assert n == mlp.n_params()
    rng = np.random.default_rng(0)
    theta = mlp.init_params(5) + 0.01 * rng.standard_normal(n)
    S.net_set_params(theta.astype(np.float32))
    theta32 = S.net_get_params().astype(np.float64)
    X = rng.standard_normal((300, 30)).astype(np.float32)
    T = rng.standard_normal((300, 27)).astype(np.float32)
    g = torch.zeros(n, dtype=torch.float32, device=DEV)
    loss = S.net_loss_grad(torch.tensor(X, device=DEV), torch.tensor(T, device=DEV), g)
    lo, go = mlp.loss_and_grad(theta32, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * lo
    gg = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gg - go) <= 1e-4 * np.linalg.norm(go)


def _training_rhs(S, j, lo=0.0, hi=1.0):
    from paper_2203_12292_amd import mfmg
    b = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    g = synth.gaussian_rhs_training(j, lo=lo, hi=hi)
    S.rhs(b, mfmg.RHS_GAUSS, g, n_terms=g.shape[0])
    return b


def test_fallback_rejects_useless_network():
    from paper_2203_12292_amd import mfmg
    S = cfg1_solver()
    S.net_set_params(np.zeros(S.net_n_params(), dtype=np.float32))
    b = _training_rhs(S, 3000)
    x_ex = torch.zeros_like(b)
    S.net_mode(mfmg.COARSE_EXACT)
    st_ex = S.solve(x_ex, b, rtol=1e-10, max_it=60, flexible=True)
    S.net_mode(mfmg.COARSE_LEARNED, tau=0.5)
    S.net_counts()
    x = torch.zeros_like(b)
    st = S.solve(x, b, rtol=1e-10, max_it=60, flexible=True)
    acc, rej, rel = S.net_counts()
    S.net_mode(mfmg.COARSE_EXACT)
    assert acc == 0 and rej == st["iterations"] and abs(rel - 1.0) < 1e-12
    assert st["iterations"] == st_ex["iterations"]
    assert (x - x_ex).abs().max().item() <= 1e-10 * x_ex.abs().max().item()


@functools.lru_cache(maxsize=None)
def gain_solver():
    from paper_2203_12292_amd import mfmg
    print("[setup] cube6 g2 ball1 Q2 (1,331 coarse DoFs)", flush=True)
    return mfmg.Solver(mfmg.Mesh(synth.CFG5_GAIN), 2)


def test_training_and_gain():
    """On a mesh whose coarse level matters (6^3 coarse cubes, 1,331 coarse
    DoFs: without any coarse correction PCG needs clearly more iterations),
    the network trained on 20,000 coarse right-hand side / exact correction
    pairs that the solver records itself needs strictly fewer iterations than
    no coarse correction, its predictions leave a smaller coarse residual
    than no correction on average, and every solve still satisfies the FP64
    oracle's equations to a relative residual of 1e-10."""
    from paper_2203_12292_amd import mfmg
    S = gain_solver()
    n_pairs = 20000
    S.net_mode(mfmg.COARSE_EXACT)
    S.net_record(n_pairs)
    x = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    j = 0
    while S.net_n_recorded() < n_pairs:
        b = _training_rhs(S, j)
        S.solve(x, b, rtol=1e-10, max_it=60)
        j += 1
    hist = S.net_train(epochs=30, batch_rows=8192, lr=2e-3, init_seed=7, shuffle_seed=11)
    print(f"[net] {S.net_n_recorded()} pairs from {j} solves, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.75 * hist[0]
    S.net_record(0)
    # validation right-hand sides (other seeds); the solutions are checked
    # against the FP64 oracle's assembled operator of this mesh
    from oracle import octree
    from oracle.space import Space, assemble_stiffness
    Sp = Space(octree.build_mesh(synth.CFG5_GAIN), 2)
    A = assemble_stiffness(Sp)
    P = perm_from_codes(Sp.codes_array(), S.dof_codes(S.n_levels - 1))
    its = {"exact": [], "learned": [], "none": [], "network alone": []}
    accepted = rejected = 0
    rels = []
    for j in range(3):
        b = _training_rhs(S, 100000 + j)
        # "network alone": every prediction accepted (no exact fallback)
        for name, mode, tau in (("exact", mfmg.COARSE_EXACT, 0.9), ("learned", mfmg.COARSE_LEARNED, 0.9),
                                ("none", mfmg.COARSE_ZERO, 0.9), ("network alone", mfmg.COARSE_LEARNED, 1e300)):
            S.net_mode(mode, tau=tau)
            S.net_counts()
            x = torch.zeros_like(b)
            st = S.solve(x, b, rtol=1e-10, max_it=200, flexible=True)
            assert st["converged"], name
            its[name].append(st["iterations"])
            if name == "learned":
                a, r, rel = S.net_counts()
                accepted += a
                rejected += r
                rels.append(rel)
            if mode == mfmg.COARSE_LEARNED:
                # final accuracy: relative residual of the oracle's equations
                bo = b.cpu().numpy()[P]
                res = np.linalg.norm(bo - A @ x.cpu().numpy()[P]) / np.linalg.norm(bo)
                assert res < 1.01e-10, (name, res)
    S.net_mode(mfmg.COARSE_EXACT)
    print(f"[net gain] iterations {its}, learned accepted {accepted} rejected {rejected}, "
          f"mean relative coarse residual {np.mean(rels):.3f} (no correction: 1, exact: 0)")
    # what the network gains over no coarse correction: fewer PCG iterations,
    # and its corrections leave a smaller coarse residual than no correction
    assert sum(its["none"]) > sum(its["exact"])
    assert sum(its["learned"]) < sum(its["none"])
    assert accepted > 0 and np.mean(rels) < 0.95


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_net_infer_matches_oracle(dtype):
    """mfmg_net_infer against the oracle's forward pass with node averaging
    and the s-scaling, element by element on every coarse DoF (shared nodes
    of 2, 4 and 8 cells; Dirichlet nodes enter as zero inputs), for fixed
    random parameters.  FP32 network arithmetic: 1e-5 of the largest entry
    (the input and output of a bfloat16 level are rounded to 8 bits: the
    oracle gets the rounded input, the output is compared at 1e-2)."""
    S = cfg1_solver()
    H = oracle_hierarchy("cfg1", 2)
    Sp = H.spaces[0]
    P0 = perm_from_codes(Sp.codes_array(), S.dof_codes(0))
    rng = np.random.default_rng(21)
    theta = mlp.init_params(13) + 0.05 * rng.standard_normal(S.net_n_params())
    S.net_set_params(theta.astype(np.float32))
    theta32 = S.net_get_params().astype(np.float64)
    for trial in range(3):
        b = rng.standard_normal(Sp.n_dofs) * (10.0 ** (trial - 1))
        g = np.zeros(len(P0))
        g[P0] = b
        bg = torch.tensor(g, dtype=dtype, device=DEV)
        yg = torch.full_like(bg, float("nan"))
        S.net_infer(yg, bg)
        torch.cuda.synchronize()
        b_used = bg.double().cpu().numpy()[P0]
        want = mlp.coarse_correction(theta32, Sp, b_used)
        got = yg.double().cpu().numpy()[P0]
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"[net infer {dtype}] trial {trial}: max error {err:.2e} of the largest entry", flush=True)
        assert err < (1e-2 if dtype == torch.bfloat16 else 1e-5), (trial, err)
    zero = torch.zeros(len(P0), dtype=dtype, device=DEV)
    y0 = torch.ones_like(zero)
    S.net_infer(y0, zero)
    torch.cuda.synchronize()
    assert float(y0.abs().max()) == 0.0


def test_net_unsupported_above_degree_two():
    """A Q3 coarse level (64 nodes per cell) has no network: the kernels hold
    nq + 3 <= 64 values per row, so set-up leaves it out and every network
    call reports MFMG_ERR_UNSUPPORTED, while the exact coarse solve works."""
    from paper_2203_12292_amd import mfmg
    print("[setup] tiny Q3 (coarse level 4^3 Q3, 1331 DoFs)", flush=True)
    S = mfmg.Solver(mfmg.Mesh(synth.CFG1_TINY), 3)
    assert S.n_dofs(0) <= 2048
    with pytest.raises(mfmg.MfmgError) as e:
        S.net_n_params()
    assert e.value.code == mfmg.ERR_UNSUPPORTED
    with pytest.raises(mfmg.MfmgError) as e:
        S.net_mode(mfmg.COARSE_LEARNED)
    assert e.value.code == mfmg.ERR_UNSUPPORTED
    b = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    S.rhs(b)
    x = torch.zeros_like(b)
    assert S.solve(x, b, rtol=1e-10, max_it=40)["converged"]
    S.close()
