"""Continuous Q_k space on a balanced octree with hanging-node and Dirichlet
constraints; assembled matrices and the intergrid prolongation (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Degrees of freedom are identified by *position*.  Each node of each leaf gets
an exact integer code per axis (``code1d``): lattice points of the finest
level (vertices, and the mid-node of an interval for even k) are one kind of
code, the other Gauss-Lobatto nodes of an interval of level l are another.
Two nodes coincide exactly when their codes are equal.

Constraints (Section 3.1: x_i = sum_j c_ij x_j + b_i, kept as constraints, not
eliminated from the mesh) are derived from their definition:

* A node on the boundary of the domain is a homogeneous Dirichlet node (its
  value is 0 and it is not a degree of freedom).
* A node of a leaf K of level l is *hanging* when it lies on the closure of a
  leaf K' of level l-1 without being one of K''s nodes.  Continuity forces its
  value to equal the interpolant of K' at that point, so c_ij = phi^{K'}_j(x_i)
  over the nodes j of K' (a node of K' is never itself hanging on a balanced
  mesh; this is asserted).
* Every other node is free.

The condensed operator is A = sum_e C_e^T A_e C_e, where C_e maps the free
DoFs to the n^3 node values of cell e (Eq. (impl:mf) with the gather G_e and
constraints C_e written as one sparse matrix), A_e the element matrix.  The
prolongation between two nested spaces (Section 3.5) is the nodal injection:
P_ij = (C_c e_j)(x_i), the coarse constrained FE function of coarse DoF j
evaluated at the fine free node x_i.  Restriction is P^T.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe
from .octree import LeafIndex

MAXLEV = 20  # finest lattice level of the codes (same constant as synth)


def bf16_round(v):
    """v rounded to the nearest bfloat16 (8 significant bits, ties to even)."""
    m, e = np.frexp(float(v))                 # v = m 2^e, 1/2 <= m < 1
    return float(np.ldexp(np.round(np.ldexp(m, 8)), e - 8))   # np.round: ties to even


def coefficient(desc):
    """c(x) of -div(c grad u) from a coefficient descriptor: kind 0 the
    constant p0 (0 -> 1); kind 1 p4 inside the ball |x - (p0,p1,p2)| <= p3,
    p5 outside; kind 2 a checkerboard of cubes of edge p2 anchored at
    (p3,p3,p3), p0 on even and p1 on odd cubes."""
    kind, p = desc["kind"], list(desc["params"]) + [0.0] * 8
    if kind == 0:
        return lambda x: p[0] if p[0] > 0 else 1.0
    if kind == 1:
        return lambda x: p[4] if sum((x[d] - p[d]) ** 2 for d in range(3)) <= p[3] ** 2 else p[5]
    if kind == 2:
        return lambda x: p[0] if sum(int(np.floor((x[d] - p[3]) / p[2])) for d in range(3)) % 2 == 0 else p[1]
    raise ValueError(kind)


def code1d(l, i, a, k):
    """Exact code of the a-th GLL node of interval i on level l."""
    if a == 0:
        return 2 * (i << (MAXLEV - l))
    if a == k:
        return 2 * ((i + 1) << (MAXLEV - l))
    if k % 2 == 0 and 2 * a == k:
        return 2 * ((2 * i + 1) << (MAXLEV - l - 1))
    return 2 * ((((l << 25) + i) * 16) + a) + 1


class CellCoefficient:
    """Cell values of a coefficient descriptor on the cells of a multigrid
    hierarchy built over the finest mesh ``fine``: a leaf of ``fine`` takes
    c at its centre; a refined cell takes the mean of its eight children's
    values (the volume average over the leaves it covers), so that coarse
    levels see the fine coefficient averaged rather than sampled.  The value
    used by the operator is this number rounded to bfloat16."""

    def __init__(self, desc, fine):
        self.c = coefficient(desc)
        self.fine = fine
        self.refined = [set(r.tolist()) for r in fine.refined]
        self.memo = {}

    def raw(self, cell):
        v = self.memo.get(cell)
        if v is None:
            l, i, j, m = cell
            if l < len(self.refined) and ((i << 42) | (j << 21) | m) in self.refined[l]:
                v = sum(self.raw((l + 1, 2 * i + a, 2 * j + b, 2 * m + c))
                        for c in (0, 1) for b in (0, 1) for a in (0, 1)) / 8.0
            else:
                h = self.fine.h(l)
                v = self.c(self.fine.lo + h * (np.array([i, j, m], float) + 0.5))
            self.memo[cell] = v
        return v

    def __call__(self, cell):
        return bf16_round(self.raw(cell))


class Space:
    """Q_k on the leaves of ``tree``; homogeneous Dirichlet on the boundary.
    ``coef``: a coefficient descriptor (None: c = 1); the operator is then
    -div(c grad u) with c constant per cell (``CellCoefficient`` over the
    finest mesh ``coef_fine``, by default ``tree`` itself)."""

    def __init__(self, tree, k, dirichlet=True, build=True, coef=None, coef_fine=None, geometry=None):
        self.tree = tree
        # mapped cells (``oracle.geometry``): a geometry descriptor, None for cubes
        self.geometry = None
        if geometry is not None and geometry["kind"] != 0:
            from .geometry import CoarseTrilinearGeometry
            self.geometry = CoarseTrilinearGeometry(tree, geometry)
        self.coef = CellCoefficient(coef, coef_fine if coef_fine is not None else tree) if coef is not None else None
        self.k = int(k)
        self.n = self.k + 1
        self.dirichlet = dirichlet
        self.index = LeafIndex(tree)
        self.xi = fe.gll_points(self.k)
        self._v1d = {}
        self._rows = {}
        self._cls = {}  # memo of classify (pure function of its arguments)
        self.cells = self.index.leaf_list()
        if build:
            self._number()

    # -- classification of nodes ------------------------------------------
    def _coarse_1d(self, s, a):
        """Coarse 1D basis values at fine node a of fine sub-interval s."""
        key = (s, a)
        v = self._v1d.get(key)
        if v is None:
            t = 0.5 * (s + self.xi[a])
            v = fe.lagrange_values(self.xi, [t])[0]
            v[np.abs(v) < 1e-14] = 0.0
            self._v1d[key] = v
        return v

    def node_code(self, cell, a, b, c):
        l, i, j, m = cell
        k = self.k
        return (code1d(l, i, a, k), code1d(l, j, b, k), code1d(l, m, c, k))

    def _on_boundary(self, cell, abc):
        l, *ijk = cell
        ext = self.tree.n0 << l
        for idx, a in zip(ijk, abc):
            if (idx == 0 and a == 0) or (idx == ext - 1 and a == self.k):
                return True
        return False

    def _coarse_candidates(self, idx, a, ext_c):
        k = self.k
        if a == 0 or a == k:
            t = idx + (1 if a == k else 0)
            cand = [t // 2] if t % 2 else [t // 2 - 1, t // 2]
        else:
            cand = [idx // 2]
        return [c for c in cand if 0 <= c < ext_c]

    def classify(self, cell, a, b, c):
        """('dir',) | ('free', code) | ('hang', coarse_cell, (vx, vy, vz))."""
        key = (cell, a, b, c)
        out = self._cls.get(key)
        if out is None:
            out = self._classify(cell, a, b, c)
            self._cls[key] = out
        return out

    def _classify(self, cell, a, b, c):
        abc = (a, b, c)
        if self.dirichlet and self._on_boundary(cell, abc):
            return ("dir",)
        l, i, j, m = cell
        code = self.node_code(cell, a, b, c)
        k = self.k
        if l == 0 or not any(x == 0 or x == k for x in abc):
            return ("free", code)
        ext_c = self.tree.n0 << (l - 1)
        cands = [self._coarse_candidates(idx, x, ext_c) for idx, x in zip((i, j, m), abc)]
        for I in cands[0]:
            for J in cands[1]:
                for M in cands[2]:
                    if not self.index.is_leaf(l - 1, I, J, M):
                        continue
                    # is the point one of the coarse cell's nodes?
                    codes_c = [set(code1d(l - 1, C, q, k) for q in range(k + 1)) for C in (I, J, M)]
                    if all(code[d] in codes_c[d] for d in range(3)):
                        return ("free", code)
                    vs = tuple(self._coarse_1d(idx - 2 * C, x)
                               for idx, C, x in zip((i, j, m), (I, J, M), abc))
                    return ("hang", (l - 1, I, J, M), vs)
        return ("free", code)

    def cell_rows(self, cell):
        """Constraint rows of a cell: list over the n^3 nodes (x fastest) of
        lists of (code, coefficient) over free DoFs."""
        r = self._rows.get(cell)
        if r is not None:
            return r
        n = self.n
        rows = []
        for c in range(n):
            for b in range(n):
                for a in range(n):
                    cl = self.classify(cell, a, b, c)
                    if cl[0] == "dir":
                        rows.append([])
                    elif cl[0] == "free":
                        rows.append([(cl[1], 1.0)])
                    else:
                        _, cc, (vx, vy, vz) = cl
                        row = []
                        for c2 in range(n):
                            if vz[c2] == 0.0:
                                continue
                            for b2 in range(n):
                                if vy[b2] == 0.0:
                                    continue
                                for a2 in range(n):
                                    if vx[a2] == 0.0:
                                        continue
                                    t = self.classify(cc, a2, b2, c2)
                                    assert t[0] != "hang", "constraint chain on a balanced mesh"
                                    if t[0] == "free":
                                        row.append((t[1], vx[a2] * vy[b2] * vz[c2]))
                        rows.append(row)
        self._rows[cell] = rows
        return rows

    def cell_has_hanging(self, cell):
        n = self.n
        for c in range(n):
            for b in range(n):
                for a in range(n):
                    if self.classify(cell, a, b, c)[0] == "hang":
                        return True
        return False

    # -- global numbering ---------------------------------------------------
    def _number(self):
        keys = set()
        for cell in self.cells:
            for row in self.cell_rows(cell):
                if len(row) == 1 and row[0][1] == 1.0:
                    keys.add(row[0][0])
        self.keys = sorted(keys)
        self.key_index = {kk: ii for ii, kk in enumerate(self.keys)}
        self.n_dofs = len(self.keys)

    def codes_array(self):
        return np.array(self.keys, dtype=np.int64).reshape(-1, 3)

    def cell_h(self, cell):
        return self.tree.h(cell[0])

    def cell_coef(self, cell):
        return 1.0 if self.coef is None else self.coef(cell)

    def element_matrix(self, cell):
        """c_e times the cell's Laplace matrix: h A_ref on a cube of side h;
        on a mapped cell, Gauss (k+1)^3 quadrature of
        |det J| (J^{-T} grad phi_i) . (J^{-T} grad phi_j) with the Jacobian
        J = dx/dxi of the cell map at every quadrature point."""
        c = self.cell_coef(cell)
        if self.geometry is None:
            return (self.cell_h(cell) * c) * fe.reference_stiffness(self.k)
        n = self.n
        xq, wq = fe.gauss(n)
        pts = np.array([(xq[a], xq[b], xq[d]) for d in range(n) for b in range(n) for a in range(n)])
        w3 = np.array([wq[a] * wq[b] * wq[d] for d in range(n) for b in range(n) for a in range(n)])
        G = fe.basis_gradient_at(self.k, pts)                 # (nq, n^3, 3) reference gradients
        J = self.geometry.jacobians(cell, pts)               # (nq, 3, 3)
        det = np.abs(np.linalg.det(J))
        phys = np.linalg.solve(np.transpose(J, (0, 2, 1)), np.transpose(G, (0, 2, 1)))  # J^T g = grad_xi
        return c * np.einsum("q,qdi,qdj->ij", w3 * det, phys, phys)

    def element_load(self, cell, f):
        """int_e f phi_i with Gauss (k+1)^3 points (|det J| weights on mapped cells)."""
        l, i, j, m = cell
        if self.geometry is None:
            h = self.cell_h(cell)
            corner = self.tree.lo + h * np.array([i, j, m], float)
            return h ** 3 * fe.reference_load(self.k, lambda xi: f(corner[None, :] + h * xi))
        n = self.n
        xq, wq = fe.gauss(n)
        pts = np.array([(xq[a], xq[b], xq[d]) for d in range(n) for b in range(n) for a in range(n)])
        w3 = np.array([wq[a] * wq[b] * wq[d] for d in range(n) for b in range(n) for a in range(n)])
        det = np.abs(np.linalg.det(self.geometry.jacobians(cell, pts)))
        return fe.basis_at(self.k, pts).T @ (w3 * det * f(self.geometry.points(cell, pts)))

    def physical_dof_points(self):
        """Coordinates of the free DoFs after the cell map (the reference
        lattice points for cubes)."""
        if self.geometry is None:
            return self.dof_points()
        out = np.zeros((self.n_dofs, 3))
        xi = self.xi
        n = self.n
        ref = np.array([(xi[a], xi[b], xi[c]) for c in range(n) for b in range(n) for a in range(n)])
        for cell in self.cells:
            pts = self.geometry.points(cell, ref)
            for q, row in enumerate(self.cell_rows(cell)):
                if len(row) == 1 and row[0][1] == 1.0:
                    out[self.key_index[row[0][0]]] = pts[q]
        return out

    def local_constraint_matrix(self, cell):
        """(global ids, dense C_e of shape (n^3, m))."""
        rows = self.cell_rows(cell)
        ids = sorted({self.key_index[kk] for row in rows for kk, _ in row})
        pos = {g: q for q, g in enumerate(ids)}
        C = np.zeros((len(rows), len(ids)))
        for r, row in enumerate(rows):
            for kk, v in row:
                C[r, pos[self.key_index[kk]]] += v
        return np.array(ids, dtype=np.int64), C

    def node_points(self, cell):
        """Physical coordinates (n^3, 3) of a cell's nodes."""
        l, i, j, m = cell
        h = self.tree.h(l)
        n = self.n
        pts = np.empty((n ** 3, 3))
        q = 0
        for c in range(n):
            for b in range(n):
                for a in range(n):
                    pts[q] = self.tree.lo + h * (np.array([i, j, m], float) + self.xi[[a, b, c]])
                    q += 1
        return pts

    def dof_points(self):
        """Coordinates of the free DoFs in the space's numbering."""
        out = np.zeros((self.n_dofs, 3))
        for cell in self.cells:
            pts = self.node_points(cell)
            for q, row in enumerate(self.cell_rows(cell)):
                if len(row) == 1 and row[0][1] == 1.0:
                    out[self.key_index[row[0][0]]] = pts[q]
        return out


# -- assembled operators -----------------------------------------------------------
def assemble_stiffness(space):
    """A = sum_e C_e^T A_e C_e as scipy CSR (n_dofs x n_dofs), A_e the
    element matrix (c_e h_e A_ref on cubes)."""
    I, J, V = [], [], []
    for cell in space.cells:
        ids, C = space.local_constraint_matrix(cell)
        if ids.size == 0:
            continue
        Al = C.T @ space.element_matrix(cell) @ C
        I.append(np.repeat(ids, ids.size))
        J.append(np.tile(ids, ids.size))
        V.append(Al.ravel())
    if not I:
        return sp.csr_matrix((space.n_dofs, space.n_dofs))
    A = sp.coo_matrix((np.concatenate(V), (np.concatenate(I), np.concatenate(J))),
                      shape=(space.n_dofs, space.n_dofs)).tocsr()
    A.sum_duplicates()
    return A


def assemble_load(space, f):
    """b = sum_e C_e^T int_e f phi, Gauss (k+1)^3; ``f`` maps (m,3) points -> (m,)."""
    b = np.zeros(space.n_dofs)
    for cell in space.cells:
        ids, C = space.local_constraint_matrix(cell)
        if ids.size == 0:
            continue
        b[ids] += C.T @ space.element_load(cell, f)
    return b


def gaussian_sum(params):
    """f(x) = sum_m a_m exp(-|x - c_m|^2 / (2 w_m^2)) for rows (cx,cy,cz,w,a)."""
    params = np.atleast_2d(params)

    def f(x):
        out = np.zeros(x.shape[0])
        for cx, cy, cz, w, a in params:
            d2 = (x[:, 0] - cx) ** 2 + (x[:, 1] - cy) ** 2 + (x[:, 2] - cz) ** 2
            out += a * np.exp(-d2 / (2.0 * w * w))
        return out
    return f


def constant(value=1.0):
    return lambda x: np.full(x.shape[0], float(value))


# -- transfer (Section 3.5) ----------------------------------------------------------
def prolongation(fine, coarse):
    """P (fine.n_dofs x coarse.n_dofs): nodal injection of the coarse space.

    The fine mesh equals the coarse mesh (polynomial coarsening) or is obtained
    from it by refining some leaves once (geometric global coarsening); every
    fine leaf is a coarse leaf or a child of one.
    """
    rows, cols, vals = [], [], []
    done = set()
    kc = coarse.k
    xic = coarse.xi
    for cell in fine.cells:
        l, i, j, m = cell
        if coarse.index.is_leaf(l, i, j, m):
            cc = cell
            shift = None
        else:
            cc = (l - 1, i >> 1, j >> 1, m >> 1)
            assert coarse.index.is_leaf(*cc), "fine leaf is neither a coarse leaf nor its child"
            shift = (i & 1, j & 1, m & 1)
        ids_c, Cc = coarse.local_constraint_matrix(cc)
        frows = fine.cell_rows(cell)
        n = fine.n
        q = 0
        for c in range(n):
            for b in range(n):
                for a in range(n):
                    row = frows[q]
                    q += 1
                    if not (len(row) == 1 and row[0][1] == 1.0):
                        continue
                    gi = fine.key_index[row[0][0]]
                    if gi in done:
                        continue
                    done.add(gi)
                    t = fine.xi[[a, b, c]]
                    if shift is not None:
                        t = 0.5 * (np.array(shift, float) + t)
                    phi = fe.basis_at(kc, t[None, :])[0]
                    val = phi @ Cc
                    nz = np.abs(val) > 1e-15
                    rows.append(np.full(int(nz.sum()), gi))
                    cols.append(ids_c[nz])
                    vals.append(val[nz])
    assert len(done) == fine.n_dofs
    if not rows:
        return sp.csr_matrix((fine.n_dofs, coarse.n_dofs))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.n_dofs, coarse.n_dofs)).tocsr()


def distribute_values(space, cell, x):
    """Node values (n^3,) of cell for the free-DoF vector x (constraints applied)."""
    ids, C = space.local_constraint_matrix(cell)
    return C @ x[ids] if ids.size else np.zeros(space.n ** 3)


def l2_error(space, x, u_exact, extra=3):
    """FE L2 error of the discrete function x against u_exact (Gauss k+1+extra)."""
    nq = space.k + 1 + extra
    xq, wq = fe.gauss(nq)
    pts = np.array([(xq[a], xq[b], xq[c]) for c in range(nq) for b in range(nq) for a in range(nq)])
    w3 = np.array([wq[a] * wq[b] * wq[c] for c in range(nq) for b in range(nq) for a in range(nq)])
    Phi = fe.basis_at(space.k, pts)
    err2 = 0.0
    for cell in space.cells:
        l, i, j, m = cell
        uh = Phi @ distribute_values(space, cell, x)
        if space.geometry is None:
            h = space.cell_h(cell)
            corner = space.tree.lo + h * np.array([i, j, m], float)
            ue = u_exact(corner[None, :] + h * pts)
            err2 += h ** 3 * np.sum(w3 * (uh - ue) ** 2)
        else:
            ue = u_exact(space.geometry.points(cell, pts))
            det = np.abs(np.linalg.det(space.geometry.jacobians(cell, pts)))
            err2 += np.sum(w3 * det * (uh - ue) ** 2)
    return np.sqrt(err2)
