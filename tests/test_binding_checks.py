"""The Python binding checks every vector argument on the host before it
becomes a raw device pointer: wrong element counts, dtypes, layouts or devices
raise before any library call (the C ABI cannot see the size of device
memory).  No GPU is needed: the library entry points are replaced by a
function that fails the test if reached."""
import numpy as np
import pytest
import torch

from paper_2203_12292_amd import mfmg


@pytest.fixture
def solver(monkeypatch):
    def no_library():
        raise AssertionError("the library was reached with a bad argument")
    monkeypatch.setattr(mfmg, "lib", no_library)
    S = object.__new__(mfmg.Solver)
    S.handle = None
    S.n_levels = 2
    S._nd = {0: 10, 1: 30, mfmg.LEVEL_ACTIVE: 30}
    return S


def test_vec_helper_order_of_checks():
    t = torch.zeros(12, dtype=torch.float64)
    with pytest.raises(TypeError):
        mfmg._vec(np.zeros(12), 12, "a")
    with pytest.raises(TypeError):
        mfmg._vec(t, 12, "a", dtype=torch.float32)
    with pytest.raises(TypeError):
        mfmg._vec(torch.zeros(12, dtype=torch.int32), 12, "a")
    with pytest.raises(ValueError, match="elements"):
        mfmg._vec(t, 13, "a")
    with pytest.raises(ValueError, match="contiguous"):
        mfmg._vec(torch.zeros(24, dtype=torch.float64)[::2], 12, "a")
    with pytest.raises(ValueError, match="GPU"):
        mfmg._vec(t, 12, "a")  # every other property is right: only the device is wrong


def test_bad_vectors_raise_before_the_library(solver):
    S = solver
    f64 = lambda n: torch.zeros(n, dtype=torch.float64)
    with pytest.raises(ValueError, match="elements"):
        S.vmult(1, f64(29), f64(30))
    with pytest.raises(TypeError):
        S.vmult(1, torch.zeros(30, dtype=torch.float32), f64(30))
    with pytest.raises(ValueError, match="elements"):
        S.vmult(1, f64(60), f64(60), n_vec=3)
    with pytest.raises(ValueError):
        S.vmult(1, f64(30), f64(30), n_vec=9)
    with pytest.raises(ValueError, match="elements"):
        S.prolongate_add(1, f64(30), f64(11))
    with pytest.raises(ValueError, match="elements"):
        S.restrict_add(1, f64(30), f64(30))
    with pytest.raises(TypeError):
        S.solve(torch.zeros(30, dtype=torch.float32), torch.zeros(30, dtype=torch.float32))
    with pytest.raises(ValueError, match="elements"):
        S.vcycle(f64(31), f64(30))
    with pytest.raises(ValueError, match="contiguous"):
        S.residual(1, f64(60)[::2], f64(30), f64(30))
    with pytest.raises(ValueError, match="reads 20"):
        S.rhs(f64(30), mfmg.RHS_GAUSS, np.zeros(15), n_terms=4)
    with pytest.raises(ValueError, match="GPU"):
        S.coarse_solve(f64(10), f64(10))
    with pytest.raises(ValueError, match="elements"):
        S.net_infer(f64(10), f64(9))


def test_set_coefficient_checks(solver):
    S = solver
    S.level_info = lambda level: {"n_cells": 7}
    with pytest.raises(ValueError, match="elements"):
        S.set_coefficient(torch.ones(8, dtype=torch.float64))
    with pytest.raises(TypeError):
        S.set_coefficient(torch.ones(7, dtype=torch.float32))
    with pytest.raises(ValueError, match="GPU"):
        S.set_coefficient(torch.ones(7, dtype=torch.float64))
