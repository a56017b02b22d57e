"""Pins of the local-smoothing oracle (Section 2.1; Algorithms 1-2, local-
smoothing branch) against facts that do not come from the oracle itself.

* On a uniformly refined mesh there is no refinement edge and every level
  covers the domain: local smoothing is then the global-coarsening V-cycle
  (itself pinned in ``test_oracle_solvers``).
* Interior level functions (zero on the refinement edge), extended by zero,
  belong to the active FE space with its hanging-node constraints and keep
  their energy: x_S^T A_SS x_S = u^T A u with u evaluated pointwise.  A wrong
  edge set or a wrong level matrix breaks this.
* The edge DoFs of level l are exactly the level-l nodes in the closure of a
  coarser leaf (checked geometrically from the leaf list).
* Galerkin identity on the refined cells: (P x)^T A^(l) (P x) equals the
  energy of x summed over the level-(l-1) cells that are refined, computed
  from element matrices.
* The V-cycle is a symmetric positive definite preconditioner, and PCG with
  it reaches the direct solution.  It needs at least as many iterations as
  global coarsening and only a few more (Section 5.2 reports a difference of
  at most one iteration on its test meshes).
"""
import functools

import numpy as np
import pytest

import synth
from oracle import fe, octree, solvers
from oracle.hierarchy import Hierarchy
from oracle.local_smoothing import LSHierarchy
from oracle.space import assemble_load, constant

from helpers import oracle_hierarchy, oracle_tree


@functools.lru_cache(maxsize=None)
def ls(name, k):
    return LSHierarchy(oracle_tree(name), k)


def eval_level_function(V, x, pts):
    """Values at ``pts`` of the level function with DoF vector x (0 outside
    the cells of the level)."""
    l = V.level
    h = V.tree.h(l)
    ext = V.tree.extent(l)
    out = np.zeros(len(pts))
    for q, p in enumerate(pts):
        c = (p - V.tree.lo) / h
        axes = []
        for v in c:
            f = int(np.floor(v + 1e-9))
            cand = [f - 1, f] if abs(v - round(v)) < 1e-9 else [f]
            axes.append([a for a in cand if 0 <= a < ext])
        for i in axes[0]:
            for j in axes[1]:
                for m in axes[2]:
                    if V.index.is_leaf(l, i, j, m):
                        ids, C = V.local_constraint_matrix((l, i, j, m))
                        t = np.clip(c - np.array([i, j, m], float), 0.0, 1.0)
                        out[q] = (fe.basis_at(V.k, t[None, :])[0] @ C) @ x[ids] if ids.size else 0.0
                        break
                else:
                    continue
                break
            else:
                continue
            break
    return out


def test_uniform_mesh_is_global_coarsening():
    desc = synth.mesh_desc("cube2_g2", 2, 0.0, 1.0, 2, [])
    tree = octree.build_mesh(desc)
    H = LSHierarchy(tree, 2)
    G = Hierarchy(tree, 2, "h")
    assert all(L.E.size == 0 for L in H.levels)
    assert [L.n for L in H.levels] == [G.levels[l].A.shape[0] for l in range(len(G.levels))]
    # the same smoother intervals on both sides
    for L, GL in zip(H.levels[1:], G.levels[1:]):
        L.smoother.lmin, L.smoother.lmax = GL.lmin, GL.lmax
    b = np.random.default_rng(3).uniform(-1, 1, H.A.shape[0])
    # the levels number their DoFs like the active space on the finest level
    fine = H.spaces[-1]
    perm = np.array([fine.key_index[kk] for kk in H.active.keys])
    lv, ac = H.maps[-1]
    assert np.array_equal(np.sort(ac), np.arange(H.A.shape[0])) and np.array_equal(perm[ac], lv)
    xg = G.vcycle(b)
    xl = H.vcycle(b)
    assert np.abs(xl - xg).max() <= 1e-12 * np.abs(xg).max()


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small_m1", 3)])
def test_interior_level_functions_extend_by_zero(name, k):
    H = ls(name, k)
    pts = H.active.dof_points()
    rng = np.random.default_rng(k)
    for L in H.levels[1:]:
        x = np.zeros(L.n)
        x[L.S] = rng.uniform(-1, 1, L.S.size)
        u = eval_level_function(L.space, x, pts)
        e_level = x[L.S] @ (L.smoother.A @ x[L.S])
        e_active = u @ (H.A @ u)
        assert abs(e_level - e_active) <= 1e-11 * e_level, L.space.level


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small", 3)])
def test_edge_dofs_are_nodes_on_coarser_leaves(name, k):
    H = ls(name, k)
    tree = oracle_tree(name)
    coarse_leaves = [(l, c) for l, c in tree.all_leaves()]
    for L in H.levels[1:]:
        V = L.space
        pts = np.zeros((V.n_dofs, 3))
        for cell in V.cells:
            for q, row in enumerate(V.cell_rows(cell)):
                if row:
                    pts[V.key_index[row[0][0]]] = V.node_points(cell)[q]
        on_coarser = np.zeros(V.n_dofs, bool)
        for l, cells in coarse_leaves:
            if l >= V.level:
                continue
            h = tree.h(l)
            lo = tree.lo + h * cells
            hi = lo + h
            inside = np.all((pts[:, None, :] >= lo[None] - 1e-12) & (pts[:, None, :] <= hi[None] + 1e-12), axis=2)
            on_coarser |= inside.any(axis=1)
        assert np.array_equal(on_coarser, V.edge), V.level


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small", 4)])
def test_galerkin_identity_on_refined_cells(name, k):
    H = ls(name, k)
    tree = oracle_tree(name)
    Aref = fe.reference_stiffness(k)
    rng = np.random.default_rng(7)
    for l in range(1, len(H.levels)):
        Vc = H.spaces[l - 1]
        xc = rng.uniform(-1, 1, Vc.n_dofs)
        xf = H.levels[l].P @ xc
        e_fine = xf @ (H.levels[l].A_full @ xf)
        e_cells = 0.0
        refined = set(tree.refined[Vc.level].tolist())
        for cell in Vc.cells:
            if int(octree.pack(*cell[1:])) not in refined:
                continue
            ids, C = Vc.local_constraint_matrix(cell)
            ue = C @ xc[ids]
            e_cells += ue @ (Vc.cell_h(cell) * Aref @ ue)
        assert abs(e_fine - e_cells) <= 1e-12 * abs(e_cells), l


@pytest.mark.parametrize("name,k", [("tiny", 1), ("small_m1", 3)])
def test_copy_maps_cover_every_active_dof_once(name, k):
    H = ls(name, k)
    seen = np.concatenate([ac for _, ac in H.maps])
    assert np.array_equal(np.sort(seen), np.arange(H.A.shape[0]))
    for (lv, ac), V in zip(H.maps, H.spaces):
        for j, i in zip(lv.tolist(), ac.tolist()):
            assert V.keys[j] == H.active.keys[i] and not V.edge[j]
    b = np.random.default_rng(0).uniform(-1, 1, H.A.shape[0])
    assert np.array_equal(H.copy_from_mg(H.copy_to_mg(b)), b)


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small_m1", 3)])
def test_vcycle_is_symmetric_positive_definite(name, k):
    H = ls(name, k)
    rng = np.random.default_rng(11)
    u, v = rng.standard_normal(H.A.shape[0]), rng.standard_normal(H.A.shape[0])
    Bu, Bv = H.vcycle(u), H.vcycle(v)
    assert abs(u @ Bv - v @ Bu) <= 1e-12 * abs(u @ Bv)
    assert u @ Bu > 0 and v @ Bv > 0


@pytest.mark.parametrize("name,k", [("tiny", 1), ("tiny", 2), ("small", 2), ("small_m1", 3)])
def test_pcg_reaches_direct_solution_with_few_more_iterations_than_gc(name, k):
    H = ls(name, k)
    G = oracle_hierarchy(name, k)
    b = assemble_load(H.active, constant(1.0))
    x, it_ls, _ = H.solve(b, rtol=1e-10)
    _, it_gc, _ = G.solve(b, rtol=1e-10)
    xd = solvers.direct_solve(H.A, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert it_gc <= it_ls <= it_gc + 3, (it_ls, it_gc)


@pytest.mark.parametrize("name,k", [("tiny", 2), ("small", 4)])
def test_polynomial_coarse_levels_variant(name, k):
    """Local smoothing down to the coarse grid, then polynomial coarsening
    there: still a symmetric positive definite preconditioner, and PCG with it
    reaches the direct solution."""
    H = LSHierarchy(oracle_tree(name), k, coarse_p=True)
    assert [L.space.k for L in H.levels[:2]] == [1, 2]
    rng = np.random.default_rng(13)
    u, v = rng.standard_normal(H.A.shape[0]), rng.standard_normal(H.A.shape[0])
    Bu, Bv = H.vcycle(u), H.vcycle(v)
    assert abs(u @ Bv - v @ Bu) <= 1e-12 * abs(u @ Bv) and u @ Bu > 0
    b = assemble_load(H.active, constant(1.0))
    x, it, _ = H.solve(b, rtol=1e-10)
    xd = solvers.direct_solve(H.A, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd) and it <= 20
