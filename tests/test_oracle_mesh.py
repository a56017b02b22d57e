"""Oracle mesh generator pinned to the counts printed in the paper.

Sources (arXiv 2203.12292): Section 4 "Examples" (octant/shell definitions and
the table of #cells, %HN and p=1 #dofs), the 1-process serial-workload columns
of the geometric multigrid statistics tables, and the exact per-level cell
counts of the single-process octant L=8 workload bar charts.  Values are stored
in tests/golden/paper_mesh_counts.json.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import octree

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_mesh_counts.json")))


def two_digits(x):
    return float(f"{x:.1e}")


@pytest.mark.parametrize("case", ["octant", "shell"])
def test_cells_dofs_workload(case):
    g = GOLD[case]
    for i, L in enumerate(g["L"]):
        if case == "octant" and L > 7:
            continue
        desc = synth.octant_mesh(L) if case == "octant" else synth.shell_mesh(L)
        t = octree.build_mesh(desc)
        assert two_digits(t.n_leaves()) == g["cells_2digit"][i], (case, L)
        assert two_digits(octree.n_vertices(t)) == g["dofs_p1_2digit"][i], (case, L)
        assert two_digits(octree.serial_workload_gc(t)) == g["wl_gc_2digit"][i], (case, L)
        assert two_digits(sum(octree.cells_per_level_ls(t))) == g["wl_ls_2digit"][i], (case, L)


@pytest.mark.parametrize("case", ["octant", "shell"])
def test_hanging_share(case):
    g = GOLD[case]
    for i, L in enumerate(g["L"]):
        desc = synth.octant_mesh(L) if case == "octant" else synth.shell_mesh(L)
        t = octree.build_mesh(desc)
        m = np.concatenate([a for _, a in octree.hanging_cell_mask(t)])
        pct = 100.0 * m.sum() / m.size
        want = g["hn_percent"][i]
        # printed with two significant digits
        assert float(f"{pct:.2g}") == want, (case, L, pct)


def test_octant_L8_levels_exact():
    t = octree.build_mesh(synth.octant_mesh(8))
    gc = [m.n_leaves() for m in octree.gc_sequence(t)][::-1]
    assert gc == GOLD["octant_L8_gc_cells_per_level"]
    assert octree.cells_per_level_ls(t) == GOLD["octant_L8_ls_cells_per_level"]


def test_closure_is_idempotent_and_balanced():
    t = octree.build_mesh(synth.CFG1)
    before = [r.copy() for r in t.refined]
    t.close()
    assert all(np.array_equal(a, b) for a, b in zip(before, t.refined))
    # brute force: any two touching leaves differ by at most one level
    leaves = [(l, c) for l, cs in t.all_leaves() for c in cs.tolist()]
    boxes = np.array([[c[0] / 2.0 ** l, c[1] / 2.0 ** l, c[2] / 2.0 ** l, 1.0 / 2.0 ** l]
                      for l, c in leaves])
    lev = np.array([l for l, _ in leaves])
    lo = boxes[:, :3]
    hi = lo + boxes[:, 3:4]
    for a in range(len(leaves)):
        touch = np.all((lo <= hi[a] + 1e-12) & (hi >= lo[a] - 1e-12), axis=1)
        assert np.all(np.abs(lev[touch] - lev[a]) <= 1)


def test_workload_meshes_sizes():
    # the benchmark meshes: ball steps towards the origin corner of [0,1]^3 (cell
    # centres within the radius), sphere-cut steps on [-1,1]^3
    seq = [m.n_leaves() for m in octree.gc_sequence(octree.build_mesh(synth.CFG1))]
    assert seq == [2808, 428, 113, 64]
    seq = [m.n_leaves() for m in octree.gc_sequence(octree.build_mesh(synth.CFG1_TINY))]
    assert seq == [386, 92, 64]


def n_dofs_entities(tree, k):
    """DoFs of a Q_k space counted per geometric entity of the leaves, as the
    paper's p=4 column counts them: every vertex, edge, face and cell of every
    leaf is one entity (a coarse face or edge next to finer leaves and the
    finer leaves' own faces and edges are different entities), carrying 1,
    k-1, (k-1)^2 and (k-1)^3 DoFs.  An entity is identified by its centre on
    the doubled finest lattice and the axes along which it extends."""
    top = tree.n_levels()
    offs = np.array([(a, b, c) for c in range(3) for b in range(3) for a in range(3)], dtype=np.int64)
    keys = {0: [], 1: [], 2: [], 3: []}
    for l, cells in tree.all_leaves():
        for off in offs:
            v = (2 * cells + off[None, :]) << (top - l)
            ext = off == 1
            keys[int(ext.sum())].append(octree.pack(v[:, 0], v[:, 1], v[:, 2]) * 8
                                        + int(ext[0]) + 2 * int(ext[1]) + 4 * int(ext[2]))
    n = {d: np.unique(np.concatenate(v)).size for d, v in keys.items()}
    assert n[3] == tree.n_leaves()
    return n[0] + (k - 1) * n[1] + (k - 1) ** 2 * n[2] + (k - 1) ** 3 * n[3]


@pytest.mark.parametrize("case", ["octant", "shell"])
def test_dofs_p4(case):
    """The p=4 DoF column of the paper's mesh table (two digits)."""
    g = GOLD[case]
    for i, L in enumerate(g["L"]):
        desc = synth.octant_mesh(L) if case == "octant" else synth.shell_mesh(L)
        t = octree.build_mesh(desc)
        assert two_digits(n_dofs_entities(t, 4)) == g["dofs_p4_2digit"][i], (case, L)
        # at p = 1 the entity count is the vertex count of the p=1 column
        assert n_dofs_entities(t, 1) == octree.n_vertices(t)
