"""The allocation-free operator entry point (mfmg_vmult_noalloc) against the
ordinary one (mfmg_vmult), through the C ABI: same kernels and inputs, so the
results agree to the last bits up to the order of the operator's LDS atomics
(FP64 1e-13, FP32 1e-6, bfloat16 one rounding of the storage type, relative to
the largest entry).  Two calls in a row share the library's fixed work space,
the second on a smaller level; a level whose work space exceeds it is refused
before any work, leaving dst untouched."""
import numpy as np
import pytest
import torch

import synth
from helpers import DESCS

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
TOL = {torch.float64: 1e-13, torch.float32: 1e-6, torch.bfloat16: 2.0 ** -7}


def rel(a, b):
    return float((a.double() - b.double()).abs().max() / b.double().abs().max())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_noalloc_matches_vmult_on_two_levels(dtype):
    from paper_2203_12292_amd import mfmg
    print(f"[setup] cfg1 Q2 and tiny Q3, {dtype}", flush=True)
    big = mfmg.Solver(mfmg.Mesh(DESCS["cfg1"]), 2, max_rhs=2)
    small = mfmg.Solver(mfmg.Mesh(DESCS["tiny"]), 3)
    rng = np.random.default_rng(3)
    for S, level, nv in ((big, big.n_levels - 1, 2), (small, small.n_levels - 1, 1)):
        n = S.n_dofs(level) * nv
        x = torch.tensor(rng.uniform(-1, 1, n), device=DEV).to(dtype)
        want = torch.empty_like(x)
        S.vmult(level, want, x, n_vec=nv)
        got = torch.full_like(x, float("nan"))
        S.vmult_noalloc(level, got, x, n_vec=nv)
        torch.cuda.synchronize()
        e = rel(got, want)
        print(f"[noalloc] {S.n_dofs(level)} DoFs x {nv}: {e:.1e}", flush=True)
        assert e <= TOL[dtype]
    big.close()
    small.close()


def test_noalloc_refuses_levels_beyond_its_work_space():
    from paper_2203_12292_amd import mfmg
    print("[setup] cube8 ball3 Q6 (more shared entries than the work space holds)", flush=True)
    S = mfmg.Solver(mfmg.Mesh(synth.ball_mesh("cube8_ball3", 8, 0, 3)), 6, mfmg.SCHEME_P_THEN_H, max_rhs=8)
    fine = S.n_levels - 1
    n = S.n_dofs(fine) * 8
    x = torch.ones(n, dtype=torch.float64, device=DEV)
    y = torch.full_like(x, 7.0)
    with pytest.raises(mfmg.MfmgError) as e:
        S.vmult_noalloc(fine, y, x, n_vec=8)
    assert e.value.code == mfmg.ERR_UNSUPPORTED and "work space" in str(e.value)
    torch.cuda.synchronize()
    assert float(y.min()) == 7.0 and float(y.max()) == 7.0
    S.close()
