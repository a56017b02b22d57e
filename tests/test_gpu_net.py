"""Learned coarse correction on the GPU.

* Gradients of the HIP forward/backward kernels (FP32) against the FP64
  oracle backward (itself checked by finite differences in
  test_oracle_mlp.py): relative error <= 1e-4.
* The exact coarse operator checks every prediction: a network that predicts 0
  is always rejected and the solve is then identical to the exact one.
* Gain: after training on coarse right-hand sides recorded from the solver,
  the learned correction is compared with the exact coarse solve and with no
  coarse correction at all; all three reach a 1e-10 relative residual in
  FP64 CG (flexible, the network makes the preconditioner non-linear).  The
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


def test_training_and_gain():
    from paper_2203_12292_amd import mfmg
    S = cfg1_solver()
    n_train = 120
    S.net_mode(mfmg.COARSE_EXACT)
    S.net_record(4000)
    x = torch.zeros(S.n_dofs(), dtype=torch.float64, device=DEV)
    for j in range(n_train):
        b = _training_rhs(S, j)
        S.solve(x, b, rtol=1e-10, max_it=60)
    n_pairs = S.net_n_recorded()
    assert n_pairs > 500
    hist = S.net_train(epochs=30, batch_rows=2048, lr=2e-3, init_seed=7, shuffle_seed=11)
    print(f"[net] {n_pairs} pairs, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.5 * hist[0]
    S.net_record(0)
    # validation right-hand sides (other seeds)
    H = oracle_hierarchy("cfg1", 2)
    P = perm_from_codes(H.spaces[-1].codes_array(), S.dof_codes(S.n_levels - 1))
    its = {"exact": [], "learned": [], "none": []}
    accepted = rejected = 0
    rels = []
    for j in range(3):
        b = _training_rhs(S, 100000 + j)
        for name, mode in (("exact", mfmg.COARSE_EXACT), ("learned", mfmg.COARSE_LEARNED),
                           ("none", mfmg.COARSE_ZERO)):
            S.net_mode(mode, tau=0.9)
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
                # final accuracy against the FP64 oracle's direct solve
                bo = b.cpu().numpy()[P]
                xo = solvers.direct_solve(H.fine.A, bo)
                err = np.linalg.norm(x.cpu().numpy()[P] - xo) / np.linalg.norm(xo)
                assert err < 1e-8, err
    S.net_mode(mfmg.COARSE_EXACT)
    print(f"[net gain] iterations {its}, learned accepted {accepted} rejected {rejected}, "
          f"mean relative coarse residual {np.mean(rels):.3f} (no correction: 1, exact: 0)")
    assert sum(its["learned"]) <= sum(its["none"])
    # what the network gains over no coarse correction: its corrections
    # leave a clearly smaller coarse residual than 1
    assert np.mean(rels) < 0.8


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
