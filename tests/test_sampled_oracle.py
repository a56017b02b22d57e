"""The sampled element-by-element evaluation (used for parity at full sizes)
against the assembled oracle matrix and load vector on small meshes, where
both fit: every free DoF of every sampled cell must match A x and b."""
import numpy as np
import pytest

import synth
from oracle.space import Space, assemble_load, assemble_stiffness, gaussian_sum

import sampled
from helpers import oracle_tree


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small", 3), ("small_m1", 2)])
def test_sampled_apply_and_load_match_assembly(name, k):
    tree = oracle_tree(name)
    S = Space(tree, k)
    A = assemble_stiffness(S)
    codes = S.codes_array()
    X = np.stack([synth.dof_hash(codes), synth.dof_hash(codes, seed=7)], axis=1)
    Y = A @ X
    params = synth.gaussian_rhs(5, 3, 0.1, 0.3, "normal", tree.lo, tree.hi)
    b = assemble_load(S, gaussian_sum(params))

    def xfun(keys):
        return np.stack([synth.dof_hash(keys), synth.dof_hash(keys, seed=7)], axis=1)

    checked = 0
    for cell in sampled.sample_cells(tree, 6, 6, seed=k):
        keys, vals = sampled.apply_at(S, cell, xfun)
        if not keys:
            continue
        ids = [S.key_index[kk] for kk in keys]
        assert np.abs(vals - Y[ids]).max() <= 1e-13 * np.abs(Y).max(), cell
        keys_b, vals_b = sampled.load_at(S, cell, [gaussian_sum(params)])
        assert keys_b == keys
        assert np.abs(vals_b[:, 0] - b[ids]).max() <= 1e-13 * np.abs(b).max(), cell
        checked += len(keys)
    assert checked > 50


def test_constrained_neighbours_are_needed():
    """Some cells have DoFs that constrain hanging nodes of leaves which do not
    touch the cell; summing over the touching leaves alone misses them."""
    from oracle import fe
    tree = oracle_tree("small")
    S = Space(tree, 2)
    A = assemble_stiffness(S)
    Y = A @ synth.dof_hash(S.codes_array())[:, None]
    Aref = fe.reference_stiffness(2)

    def local(c, rows):
        u = np.array([[sum(w * synth.dof_hash(np.array([kk]))[0] for kk, w in row)] for row in rows])
        return S.cell_h(c) * (Aref @ u)

    needed = 0
    for cell in S.cells:
        keys = sampled.own_dofs(S, cell)
        if not keys:
            continue
        ids = [S.key_index[kk] for kk in keys]
        direct = []
        for lv in range(max(0, cell[0] - 1), cell[0] + 2):
            direct += sampled._touching(S, lv, cell)
        full = sampled.neighbourhood(S, cell)
        assert set(direct) <= set(full)
        extra = [c for c in full if c not in set(direct)]
        if not extra:
            continue
        assert np.abs(sampled._accumulate(S, full, keys, local) - Y[ids]).max() < 1e-13 * np.abs(Y).max()
        part = sampled._accumulate(S, direct, keys, local)
        if np.abs(part - Y[ids]).max() > 1e-6 * np.abs(Y).max():
            needed += 1
            if needed >= 3:
                break
    assert needed >= 3
