"""Element-by-element oracle evaluation of single output entries on meshes too
large to assemble (test infrastructure).

For a sampled cell e, every free DoF i that is a node of e receives
contributions (C_c^T A_c C_c x)_i only from leaves c whose constrained node
rows involve i (Eq. (impl:mf) with C_c the constraint matrix of cell c):

* leaves that contain the node of i, which touch e and are at most one level
  coarser or finer than e on a one-irregular mesh;
* leaves with hanging nodes constrained by i, which lie one level below a
  leaf E that contains the node of i and touch E.

``neighbourhood`` returns a superset of these leaves; summing over it gives
the exact entry.  DoFs are identified by their exact position codes.
"""
from __future__ import annotations

import numpy as np

from oracle import fe, octree


def _touching(space, lv, cell):
    """Leaves of level lv whose closure meets the closure of ``cell``."""
    L, i, j, m = cell
    ext = space.tree.n0 << lv
    if lv >= L:
        s = 1 << (lv - L)
        rng = [range(max(0, a * s - 1), min(ext, (a + 1) * s + 1)) for a in (i, j, m)]
    else:
        s = L - lv
        rng = [range(max(0, (a >> s) - 1), min(ext, (a >> s) + 2)) for a in (i, j, m)]
    out = []
    for a in rng[0]:
        for b in rng[1]:
            for c in rng[2]:
                if space.index.is_leaf(lv, a, b, c):
                    out.append((lv, a, b, c))
    return out


def neighbourhood(space, cell):
    """A superset of the leaves that contribute to the free DoFs of ``cell``."""
    L = cell[0]
    top = space.tree.n_levels()  # leaves can sit one level below the last refined one
    direct = []
    for lv in range(max(0, L - 1), min(top, L + 1) + 1):
        direct += _touching(space, lv, cell)
    out = set(direct)
    for E in direct:
        if E[0] + 1 <= top:
            out.update(_touching(space, E[0] + 1, E))
    return sorted(out)


def own_dofs(space, cell):
    """Codes of the free DoFs that are nodes of ``cell``."""
    keys = []
    for row in space.cell_rows(cell):
        if len(row) == 1 and row[0][1] == 1.0:
            keys.append(row[0][0])
    return keys


def _accumulate(space, cells, targets, local):
    """sum over cells c of C_c^T local(c) restricted to the target codes."""
    pos = {kk: q for q, kk in enumerate(targets)}
    out = None
    for c in cells:
        rows = space.cell_rows(c)
        if not any(kk in pos for row in rows for kk, _ in row):
            continue
        v = local(c, rows)
        if out is None:
            out = np.zeros((len(targets),) + v.shape[1:])
        for q, row in enumerate(rows):
            for kk, w in row:
                t = pos.get(kk)
                if t is not None:
                    out[t] += w * v[q]
    return out


def apply_at(space, cell, xfun):
    """(codes, values) of (A x) at the free DoFs of ``cell``; ``xfun`` maps an
    (m, 3) int64 code array to the (m, nv) input values."""
    targets = own_dofs(space, cell)
    cells = neighbourhood(space, cell)
    Aref = fe.reference_stiffness(space.k)
    cache = {}

    def local(c, rows):
        keys = sorted({kk for row in rows for kk, _ in row})
        missing = [kk for kk in keys if kk not in cache]
        if missing:
            vals = xfun(np.array(missing, dtype=np.int64).reshape(-1, 3))
            for kk, v in zip(missing, vals):
                cache[kk] = v
        nv = next(iter(cache.values())).shape[0] if cache else 1
        u = np.zeros((len(rows), nv))
        for q, row in enumerate(rows):
            for kk, w in row:
                u[q] += w * cache[kk]
        return (space.cell_h(c) * space.cell_coef(c)) * (Aref @ u)

    return targets, _accumulate(space, cells, targets, local)


def load_at(space, cell, fs):
    """(codes, values) of the load vectors b = sum_e C_e^T int_e f phi at the
    free DoFs of ``cell``, one column per function in ``fs``."""
    targets = own_dofs(space, cell)
    cells = neighbourhood(space, cell)
    k = space.k

    def local(c, rows):
        l, i, j, m = c
        h = space.cell_h(c)
        corner = space.tree.lo + h * np.array([i, j, m], float)
        return np.stack([h ** 3 * fe.reference_load(k, lambda xi: f(corner[None, :] + h * xi)) for f in fs],
                        axis=1)

    return targets, _accumulate(space, cells, targets, local)


def sample_cells(tree, n_plain, n_hanging, seed):
    """Random leaves, ``n_hanging`` of them with hanging nodes."""
    rng = np.random.default_rng(seed)
    per_level = tree.all_leaves()
    lev = np.concatenate([np.full(c.shape[0], l) for l, c in per_level])
    ijk = np.concatenate([c for _, c in per_level])
    hang = np.concatenate([m for _, m in octree.hanging_cell_mask(tree)])
    hang_idx = np.flatnonzero(hang)
    plain = rng.choice(lev.size, size=n_plain, replace=False)
    hanging = rng.choice(hang_idx, size=min(n_hanging, hang_idx.size), replace=False)
    return [(int(lev[q]), *(int(v) for v in ijk[q])) for q in np.concatenate([plain, hanging])]


def locate(codes, hashes, keys, key_hash):
    """Positions in the library's numbering of the DoFs with codes ``keys``,
    found through a per-DoF hash value (checked against the full codes)."""
    want = key_hash(np.array(keys, dtype=np.int64).reshape(-1, 3))
    # hashes lie in [-1, 1): bucket them on a 2^21 grid, then compare exactly
    bucket = ((hashes + 1.0) * 2.0 ** 20).astype(np.int64)
    cand = np.flatnonzero(np.isin(bucket, ((want + 1.0) * 2.0 ** 20).astype(np.int64), kind="table"))
    wanted = set(want.tolist())
    by_hash = {}
    for p in cand.tolist():
        if hashes[p] in wanted:
            by_hash.setdefault(hashes[p], []).append(p)
    out = []
    for kk, hv in zip(keys, want.tolist()):
        cands = [p for p in by_hash.get(hv, []) if tuple(codes[p]) == tuple(kk)]
        assert len(cands) == 1, kk
        out.append(cands[0])
    return np.array(out, dtype=np.int64)
