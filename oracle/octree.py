"""Octree meshes of the unit-cube family, closure and global coarsening (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A mesh is a forest over an ``n0^3`` grid of coarse cubes.  A cell at level l
is the integer triple (i, j, k) with 0 <= i, j, k < n0 * 2^l.  The tree is
stored as the set of *refined* cells per level; a cell exists when its parent
is refined (level 0 cells always exist) and is a leaf when it exists and is
not refined.

* Refinement steps and the closure follow the construction of the paper's test
  meshes (Section 4, "Examples"): mark cells by a criterion on the cell centre,
  refine, then close so that leaves which touch differ by at most one level.
* The global-coarsening level sequence follows Section 2.2: all cells are
  coarsened simultaneously (every refined cell whose children are all leaves
  loses its children), then the closure is applied again; repeat until only
  the coarse grid remains.
"""
from __future__ import annotations

import numpy as np

import synth

_B = 21
_MASK = (1 << _B) - 1
_OFFS26 = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)
                    if (a, b, c) != (0, 0, 0)], dtype=np.int64)
_CHILD8 = np.array([(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.int64)


def pack(i, j, k):
    return (np.asarray(i, np.int64) << 42) | (np.asarray(j, np.int64) << 21) | np.asarray(k, np.int64)


def unpack(key):
    key = np.asarray(key, np.int64)
    return (key >> 42) & _MASK, (key >> 21) & _MASK, key & _MASK


def _unpack3(key):
    i, j, k = unpack(key)
    return np.stack([i, j, k], axis=-1)


class Octree:
    def __init__(self, n0, lo=0.0, hi=1.0):
        self.n0 = int(n0)
        self.lo = float(lo)
        self.hi = float(hi)
        self.refined = [np.zeros(0, np.int64)]

    # -- structure ---------------------------------------------------------
    def copy(self):
        t = Octree(self.n0, self.lo, self.hi)
        t.refined = [r.copy() for r in self.refined]
        return t

    def n_levels(self):
        return len(self.refined)

    def extent(self, level):
        return self.n0 << level

    def h(self, level):
        return (self.hi - self.lo) / (self.n0 * 2.0 ** level)

    def existing(self, level):
        if level == 0:
            n = self.n0
            g = np.arange(n, dtype=np.int64)
            i, j, k = np.meshgrid(g, g, g, indexing="ij")
            return np.sort(pack(i.ravel(), j.ravel(), k.ravel()))
        par = self.refined[level - 1]
        if par.size == 0:
            return np.zeros(0, np.int64)
        p = _unpack3(par)
        ch = (2 * p[:, None, :] + _CHILD8[None, :, :]).reshape(-1, 3)
        return np.sort(pack(ch[:, 0], ch[:, 1], ch[:, 2]))

    def leaves(self, level):
        ex = self.existing(level)
        if level < len(self.refined):
            return np.setdiff1d(ex, self.refined[level], assume_unique=True)
        return ex

    def all_leaves(self):
        """List of (level, int64 array (m, 3)) for every level with leaves."""
        out = []
        for l in range(len(self.refined) + 1):
            lv = self.leaves(l)
            if lv.size:
                out.append((l, _unpack3(lv)))
        return out

    def n_leaves(self):
        return sum(a.shape[0] for _, a in self.all_leaves())

    def _add_refined(self, level, keys):
        while len(self.refined) <= level + 1:
            self.refined.append(np.zeros(0, np.int64))
        self.refined[level] = np.union1d(self.refined[level], keys)

    def _trim(self):
        while len(self.refined) > 1 and self.refined[-1].size == 0:
            self.refined.pop()

    # -- closure -----------------------------------------------------------
    def close(self):
        """One-irregularity closure.

        For every refined cell P at level l >= 1, each of its 26 same-level
        neighbours inside the domain must exist, i.e. the neighbour's parent
        must be refined.  Sweeping from the finest level downwards settles
        everything in one pass (new refinements at level l-1 are inspected
        when the sweep reaches l-1).
        """
        for l in range(len(self.refined) - 1, 0, -1):
            P = self.refined[l]
            if P.size == 0:
                continue
            c = _unpack3(P)
            q = (c[:, None, :] + _OFFS26[None, :, :]).reshape(-1, 3)
            n = self.extent(l)
            ok = np.all((q >= 0) & (q < n), axis=1)
            q = q[ok] >> 1
            need = np.unique(pack(q[:, 0], q[:, 1], q[:, 2]))
            self._add_refined(l - 1, need)
        self._trim()

    # -- refinement by a criterion ----------------------------------------
    def centres(self, level, cells):
        h = (self.hi - self.lo) / (self.n0 * 2.0 ** level)
        return self.lo + (cells.astype(np.float64) + 0.5) * h

    def _mark(self, level, cells, kind, params):
        h = (self.hi - self.lo) / (self.n0 * 2.0 ** level)
        c = self.lo + (cells.astype(np.float64) + 0.5) * h
        if kind == synth.ALL:
            return np.ones(cells.shape[0], bool)
        if kind == synth.BALL:
            x0, y0, z0, r = params[:4]
            d2 = (c[:, 0] - x0) ** 2 + (c[:, 1] - y0) ** 2 + (c[:, 2] - z0) ** 2
            return d2 <= r * r
        if kind == synth.BOX_LE:
            a, b, cc = params[:3]
            return (c[:, 0] <= a) & (c[:, 1] <= b) & (c[:, 2] <= cc)
        if kind == synth.BAND:
            x0, y0, z0, r1, r2 = params[:5]
            d2 = (c[:, 0] - x0) ** 2 + (c[:, 1] - y0) ** 2 + (c[:, 2] - z0) ** 2
            return (d2 >= r1 * r1) & (d2 <= r2 * r2)
        if kind == synth.SPHERE_CUT:
            x0, y0, z0, ra, rb = params[:5]
            lo = self.lo + cells.astype(np.float64) * h
            hi = self.lo + (cells.astype(np.float64) + 1.0) * h
            ctr = np.array([x0, y0, z0])
            near = np.clip(ctr[None, :], lo, hi)
            dmin2 = np.sum((near - ctr[None, :]) ** 2, axis=1)
            far = np.where(np.abs(lo - ctr) > np.abs(hi - ctr), lo, hi)
            dmax2 = np.sum((far - ctr[None, :]) ** 2, axis=1)
            m = (dmin2 <= ra * ra) & (ra * ra <= dmax2)
            if rb > 0:
                m |= (dmin2 <= rb * rb) & (rb * rb <= dmax2)
            return m
        raise ValueError(f"unknown predicate kind {kind}")

    def refine_where(self, kind, params):
        for l, cells in self.all_leaves():
            m = self._mark(l, cells, kind, params)
            if np.any(m):
                sel = cells[m]
                self._add_refined(l, pack(sel[:, 0], sel[:, 1], sel[:, 2]))
        self.close()

    # -- global coarsening (Section 2.2) ------------------------------------
    def coarsened(self):
        """Next coarser level: drop every terminal family, then close again."""
        t = self.copy()
        for l in range(len(t.refined)):
            R = t.refined[l]
            if R.size == 0:
                continue
            if l + 1 < len(t.refined) and t.refined[l + 1].size:
                q = _unpack3(t.refined[l + 1]) >> 1
                nonterminal = np.unique(pack(q[:, 0], q[:, 1], q[:, 2]))
            else:
                nonterminal = np.zeros(0, np.int64)
            # only cells of R with a refined child survive
            t.refined[l] = np.intersect1d(R, nonterminal, assume_unique=True)
        t._trim()
        t.close()
        return t

    def is_coarse_grid(self):
        return all(r.size == 0 for r in self.refined)


def build_mesh(desc):
    """Octree for a ``synth`` mesh descriptor."""
    t = Octree(desc["n0"], desc["lo"], desc["hi"])
    for _ in range(desc["n_global"]):
        t.refine_where(synth.ALL, ())
    for kind, params in desc["steps"]:
        t.refine_where(kind, params)
    return t


def gc_sequence(tree):
    """Global-coarsening meshes, finest first, ending at the coarse grid."""
    seq = [tree]
    while not seq[-1].is_coarse_grid():
        seq.append(seq[-1].coarsened())
    return seq


class LeafIndex:
    """Fast leaf membership for a mesh: set of (level, i, j, k)."""

    def __init__(self, tree):
        self.tree = tree
        self.keys = {}
        for l, cells in tree.all_leaves():
            self.keys[l] = set(pack(cells[:, 0], cells[:, 1], cells[:, 2]).tolist())

    def is_leaf(self, l, i, j, k):
        s = self.keys.get(l)
        return s is not None and ((i << 42) | (j << 21) | k) in s

    def leaf_list(self):
        """Leaves as a list of (l, i, j, k), coarse-to-fine, lexicographic."""
        out = []
        for l, cells in self.tree.all_leaves():
            for c in cells.tolist():
                out.append((l, c[0], c[1], c[2]))
        return out

    def find_leaf(self, l, i, j, k):
        """Leaf containing level-l cell (i,j,k) (an ancestor or itself), or None."""
        for m in range(l, -1, -1):
            s = l - m
            if self.is_leaf(m, i >> s, j >> s, k >> s):
                return (m, i >> s, j >> s, k >> s)
        return None


# -- mesh statistics (Section 4 metrics) -------------------------------------------
_OFFS18 = np.array([o for o in _OFFS26.tolist() if sum(1 for v in o if v != 0) <= 2], dtype=np.int64)


def hanging_cell_mask(tree):
    """Per level, a boolean array over that level's leaves: does the leaf carry
    hanging-node constraints?  A leaf of level l has hanging nodes exactly when
    one of the level-l cells sharing a face or an edge with it lies inside the
    domain but does not exist (it is covered by a coarser leaf)."""
    out = []
    for l, cells in tree.all_leaves():
        if l == 0:
            out.append((l, np.zeros(cells.shape[0], bool)))
            continue
        q = cells[:, None, :] + _OFFS18[None, :, :]
        n = tree.extent(l)
        inside = np.all((q >= 0) & (q < n), axis=2)
        par = q >> 1
        pk = pack(par[..., 0], par[..., 1], par[..., 2])
        exists = np.isin(pk, tree.refined[l - 1])
        out.append((l, np.any(inside & ~exists, axis=1)))
    return out


def n_vertices(tree):
    """Number of distinct cell vertices (the DoFs of a Q1 space counted with
    constrained and boundary ones, as the paper's p=1 column counts them)."""
    top = tree.n_levels()
    keys = []
    for l, cells in tree.all_leaves():
        s = top - l
        for off in _CHILD8:
            v = (cells + off[None, :]) << s
            keys.append(pack(v[:, 0], v[:, 1], v[:, 2]))
    return int(np.unique(np.concatenate(keys)).size)


def serial_workload_gc(tree):
    """W_s = sum over the global-coarsening levels of their cell counts."""
    return sum(m.n_leaves() for m in gc_sequence(tree))


def cells_per_level_ls(tree):
    """Cells of each refinement level (active or not), the local-smoothing levels."""
    return [tree.existing(l).size for l in range(tree.n_levels() + 1)]
