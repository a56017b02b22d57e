"""Q_k Lagrange elements on hexahedra (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Nodes: Gauss-Lobatto-Legendre points of degree k on [0, 1] (the paper uses
  tensor products of 1D Lagrange elements of degree p; the node family is our
  reading, the FE space does not depend on it).
* Quadrature: Gauss-Legendre with (k+1) points per direction, (k+1)^3 in 3D
  (Section 5 set-up: "consistent Gauss-Legendre quadrature with (p+1)^3
  points").
* Local numbering is lexicographic with x fastest: node (a, b, c) has index
  a + n*b + n*n*c, n = k+1.

Element matrices are built the textbook way: the gradients of all n^3 basis
functions are tabulated at all n^3 quadrature points and A_e = sum_q w_q
grad(phi_i)(x_q) . grad(phi_j)(x_q) |det J|.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(k):
    """Gauss-Lobatto-Legendre points of degree k, mapped to [0, 1]."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if k == 1:
        return np.array([0.0, 1.0])
    # interior GLL points are the roots of P_k'
    coef = np.zeros(k + 1)
    coef[k] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(coef)).real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    # symmetrise to remove root-finder asymmetry
    x = 0.5 * (x - x[::-1])
    return 0.5 * (x + 1.0)


def gauss(n):
    """n-point Gauss-Legendre rule on [0, 1]: points, weights."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """V[q, i] = l_i(x_q) for the Lagrange polynomials on ``nodes``."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = nodes.size
    V = np.ones((x.size, n))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[q, i] = l_i'(x_q) (product rule, term by term)."""
    nodes = np.asarray(nodes, float)
    x = np.atleast_1d(np.asarray(x, float))
    n = nodes.size
    D = np.zeros((x.size, n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(x.size, 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D


def tensor3(Az, Ay, Ax):
    """3D tabulation from 1D ones for lexicographic (x fastest) ordering."""
    return np.kron(Az, np.kron(Ay, Ax))


def reference_stiffness(k):
    """Laplace element matrix on the unit cube [0,1]^3, Gauss (k+1)^3 points."""
    nodes = gll_points(k)
    xq, wq = gauss(k + 1)
    V = lagrange_values(nodes, xq)
    D = lagrange_derivatives(nodes, xq)
    w3 = tensor3(wq[:, None], wq[:, None], wq[:, None]).ravel()
    grads = [tensor3(V, V, D), tensor3(V, D, V), tensor3(D, V, V)]
    return sum(G.T @ (w3[:, None] * G) for G in grads)


def element_stiffness(k, h):
    """Laplace element matrix on an axis-aligned cube of side h.

    With x = x0 + h xi: grad = grad_xi / h and |det J| = h^3, so the matrix is
    h * reference_stiffness(k).
    """
    return h * reference_stiffness(k)


def reference_load(k, f_ref):
    """Load vector int_{[0,1]^3} f(xi) phi_i(xi) with Gauss (k+1)^3 points.

    ``f_ref``: callable taking an (nq, 3) array of reference points.
    """
    nodes = gll_points(k)
    xq, wq = gauss(k + 1)
    V = lagrange_values(nodes, xq)
    n = k + 1
    pts = np.array([(xq[a], xq[b], xq[c]) for c in range(n) for b in range(n) for a in range(n)])
    w3 = tensor3(wq[:, None], wq[:, None], wq[:, None]).ravel()
    return tensor3(V, V, V).T @ (w3 * f_ref(pts))


def basis_at(k, xi):
    """Values of all n^3 basis functions at reference points xi (m, 3)."""
    nodes = gll_points(k)
    xi = np.atleast_2d(xi)
    Vx = lagrange_values(nodes, xi[:, 0])
    Vy = lagrange_values(nodes, xi[:, 1])
    Vz = lagrange_values(nodes, xi[:, 2])
    n = k + 1
    out = np.empty((xi.shape[0], n ** 3))
    for c in range(n):
        for b in range(n):
            for a in range(n):
                out[:, a + n * b + n * n * c] = Vx[:, a] * Vy[:, b] * Vz[:, c]
    return out


def basis_gradient_at(k, xi):
    """Reference gradients (m, n^3, 3) of all basis functions at points xi."""
    nodes = gll_points(k)
    xi = np.atleast_2d(xi)
    V = [lagrange_values(nodes, xi[:, d]) for d in range(3)]
    D = [lagrange_derivatives(nodes, xi[:, d]) for d in range(3)]
    n = k + 1
    out = np.empty((xi.shape[0], n ** 3, 3))
    for c in range(n):
        for b in range(n):
            for a in range(n):
                i = a + n * b + n * n * c
                out[:, i, 0] = D[0][:, a] * V[1][:, b] * V[2][:, c]
                out[:, i, 1] = V[0][:, a] * D[1][:, b] * V[2][:, c]
                out[:, i, 2] = V[0][:, a] * V[1][:, b] * D[2][:, c]
    return out
