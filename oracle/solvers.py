"""Chebyshev-Jacobi smoothing, the global-coarsening V-cycle and PCG (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Smoother (Section 3.3): Chebyshev iteration around point Jacobi, i.e. the
  Chebyshev acceleration of x <- x + D^{-1}(b - A x) (Saad, Iterative Methods
  for Sparse Linear Systems, 2nd ed., Algorithm 12.1, applied to D^{-1}A).
  Degree m means m updates of x; from x = 0 the first update needs no
  operator evaluation, so degree 3 costs 2 evaluations before the coarse
  correction and 3 after it, as the paper counts them (Section 5.1).
* The eigenvalue interval [lambda_max/20, 1.2 lambda_max] with lambda_max
  estimated by 15 steps of Jacobi-preconditioned CG started from b = 1
  (the Lanczos tridiagonal matrix built from the CG coefficients).
* V-cycle (Algorithms 1-2, global-coarsening branch, A^(l) = A_SS^(l)).
* CG preconditioned by one V-cycle per iteration (Section 2), x0 = 0, stopped
  on the l2 norm of the unpreconditioned residual relative to ||b||.
* Full multigrid (textbook; named by the paper as a benefit of global
  coarsening).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def estimate_lambda_max(A, Dinv, n_iter=15):
    """Largest eigenvalue estimate of D^{-1}A from CG's Lanczos coefficients."""
    n = A.shape[0]
    if n == 0:
        return 1.0
    b = np.ones(n)
    x = np.zeros(n)
    r = b.copy()
    z = Dinv * r
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(min(n_iter, n)):
        Ap = A @ p
        pAp = p @ Ap
        if pAp <= 0.0 or rz <= 0.0:
            break
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        z = Dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        rz = rz_new
        if rz <= 0.0:
            break
        p = z + beta * p
    m = len(alphas)
    if m == 0:
        return 1.0
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return float(np.max(np.linalg.eigvalsh(T)))


def chebyshev_interval(lambda_max_est, smoothing_range=20.0, safety=1.2):
    lmax = safety * lambda_max_est
    return lmax / smoothing_range, lmax


def chebyshev(A, Dinv, b, x0, degree, lmin, lmax):
    """Chebyshev acceleration of Jacobi; ``x0=None`` means x0 = 0."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b.copy() if x0 is None else b - A @ x
    d = (Dinv * r) / theta
    x = x + d
    for _ in range(degree - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        r = b - A @ x
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (Dinv * r)
        x = x + d
        rho = rho_new
    return x


class Level:
    def __init__(self, A, P=None, degree=3):
        self.A = A.tocsr()
        self.diag = self.A.diagonal().copy()
        self.Dinv = np.where(self.diag > 0, 1.0 / np.where(self.diag > 0, self.diag, 1.0), 0.0)
        self.P = P  # prolongation from the next coarser level (None on level 0)
        self.degree = degree
        self.lmin = self.lmax = None

    def setup_smoother(self, n_iter=15):
        lam = estimate_lambda_max(self.A, self.Dinv, n_iter)
        self.lmin, self.lmax = chebyshev_interval(lam)


class CoarseDirect:
    """Exact coarse-grid solver (dense Cholesky of A^(0))."""

    def __init__(self, A0):
        n = A0.shape[0]
        self.n = n
        if n:
            self.factor = sla.cho_factor(A0.toarray())

    def __call__(self, b):
        if self.n == 0:
            return b.copy()
        return sla.cho_solve(self.factor, b)


def vcycle(levels, b, coarse_solver, l=None):
    """Algorithm 2 (global coarsening) on levels[0..L], returning x^(l)."""
    if l is None:
        l = len(levels) - 1
    if l == 0:
        return coarse_solver(b)
    L = levels[l]
    x = chebyshev(L.A, L.Dinv, b, None, L.degree, L.lmin, L.lmax)      # presmoothing
    r = b - L.A @ x                                                     # residual
    bc = np.zeros(levels[l - 1].A.shape[0]) + L.P.T @ r                 # restrict-add
    xc = vcycle(levels, bc, coarse_solver, l - 1)                       # recursion
    x = x + L.P @ xc                                                    # prolongate-add
    x = chebyshev(L.A, L.Dinv, b, x, L.degree, L.lmin, L.lmax)          # postsmoothing
    return x


def fmg(levels, b, coarse_solver, cycles=1):
    """Full multigrid with V-cycles (textbook form: Trottenberg, Oosterlee,
    Schueller, Multigrid, 2001, Sec. 2.6), which the paper names as a solver
    that global coarsening makes easy to build (Section 2.2).

    The right-hand side is carried to every level by the restriction,
    b^(l-1) = P^T b^(l); the coarsest level is solved exactly; then on each
    finer level the prolongated coarse result is the initial guess and
    ``cycles`` V-cycles correct it, x <- x + V(b - A x).
    """
    bs = [None] * len(levels)
    bs[-1] = b
    for l in range(len(levels) - 1, 0, -1):
        bs[l - 1] = levels[l].P.T @ bs[l]
    x = coarse_solver(bs[0])
    for l in range(1, len(levels)):
        x = levels[l].P @ x
        for _ in range(cycles):
            x = x + vcycle(levels, bs[l] - levels[l].A @ x, coarse_solver, l)
    return x


def pcg(A, b, precond, rtol=1e-10, max_it=500, flexible=False):
    """CG with a preconditioner; returns x, iterations, residual history."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return x, 0, hist
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, max_it + 1):
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r_old_z = z
        r -= alpha * Ap
        res = np.linalg.norm(r) / nb
        hist.append(res)
        if res <= rtol:
            return x, it, hist
        z = precond(r)
        rz_new = r @ z
        beta = ((rz_new - r @ r_old_z) / rz) if flexible else (rz_new / rz)
        rz = rz_new
        p = z + beta * p
    return x, max_it, hist


def direct_solve(A, b):
    return spla.spsolve(A.tocsc(), b)
