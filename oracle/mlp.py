"""Per-coarse-cell network of the learned coarse correction (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The coarse-grid solve of Algorithm 2 (level 0) is replaced by a small
multilayer perceptron evaluated independently on every coarse cell:

* input (30): the coarse right-hand side at the cell's 27 nodes (Q2 on the
  coarse grid), divided by s = ||b^(0)||_2, and the 3 coordinates of the cell
  centre;
* two hidden layers of width 64 with GELU(z) = z Phi(z) (Phi the standard
  normal distribution function), then a linear output layer of 27;
* output: the correction at the cell's 27 nodes divided by s; nodes shared by
  several cells average the cells' predictions, Dirichlet nodes are 0.

Training minimises the mean squared error to the exact coarse solution
A^(0)^{-1} b^(0) (same scaling) with Adam (Kingma & Ba, 2015).  Parameters
are stored flat in the order W1 (30x64, row-major), b1, W2 (64x64), b2,
W3 (64x27), b3.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SIZES = (30, 64, 64, 27)


def n_params(sizes=SIZES):
    return sum(sizes[i] * sizes[i + 1] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(theta, sizes=SIZES):
    out, p = [], 0
    for i in range(len(sizes) - 1):
        a, b = sizes[i], sizes[i + 1]
        W = theta[p:p + a * b].reshape(a, b)
        p += a * b
        bias = theta[p:p + b]
        p += b
        out.append((W, bias))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def sizes_for(nin):
    """Layer widths for nin inputs: the nq = nin - 3 node values and 3 centre
    coordinates in, two hidden layers of 64, nq outputs."""
    return (nin, 64, 64, nin - 3)


def forward(theta, X):
    """Y (rows x nq) and the cache of pre-activations (nq = X.shape[1] - 3)."""
    X = np.asarray(X, dtype=np.float64)
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta, sizes_for(X.shape[1]))
    Z1 = X @ W1 + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2)
    Y = H2 @ W3 + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(theta, X, T):
    """Mean squared error over all rows and outputs."""
    Y, _ = forward(theta, X)
    return float(np.mean((Y - T) ** 2))


def loss_and_grad(theta, X, T):
    """Loss and its gradient w.r.t. theta (reverse-mode chain rule)."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta, sizes_for(np.shape(X)[1]))
    Y, (X, Z1, H1, Z2, H2) = forward(theta, X)
    n = Y.size
    D3 = 2.0 * (Y - T) / n
    gW3 = H2.T @ D3
    gb3 = D3.sum(axis=0)
    D2 = (D3 @ W3.T) * gelu_prime(Z2)
    gW2 = H1.T @ D2
    gb2 = D2.sum(axis=0)
    D1 = (D2 @ W2.T) * gelu_prime(Z1)
    gW1 = X.T @ D1
    gb1 = D1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.mean((Y - T) ** 2)), g


class Adam:
    """Adam with bias correction."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def init_params(seed=0, sizes=SIZES):
    """He-style initialisation (normal, std sqrt(2/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        a, b = sizes[i], sizes[i + 1]
        parts.append(rng.standard_normal(a * b) * np.sqrt(2.0 / a))
        parts.append(np.zeros(b))
    return np.concatenate(parts)


def coarse_correction(theta, space, b):
    """The network's coarse correction y for the right-hand side b of the
    coarse space ``space`` (a conforming mesh: no hanging nodes).

    With s = ||b||_2, each leaf cell is one row of the network: inputs the
    values of b at the cell's (k+1)^3 nodes (x fastest; 0 at Dirichlet nodes)
    divided by s, then the cell centre; outputs the cell's nodal correction
    divided by s.  A DoF takes s times the mean of the outputs of the cells
    that have it as a node.  b = 0 gives y = 0.
    """
    b = np.asarray(b, dtype=np.float64)
    s = float(np.linalg.norm(b))
    y = np.zeros(space.n_dofs)
    if s == 0.0:
        return y
    count = np.zeros(space.n_dofs)
    for cell in space.cells:
        ids = []
        for row in space.cell_rows(cell):
            if not row:
                ids.append(-1)  # Dirichlet node
                continue
            assert len(row) == 1 and row[0][1] == 1.0, "coarse space with hanging nodes"
            ids.append(space.key_index[row[0][0]])
        ids = np.array(ids)
        l, i, j, m = cell
        centre = space.tree.lo + space.tree.h(l) * (np.array([i, j, m], float) + 0.5)
        x = np.concatenate([np.where(ids >= 0, b[np.maximum(ids, 0)], 0.0) / s, centre])
        out = forward(theta, x[None, :])[0][0]
        for q, g in enumerate(ids):
            if g >= 0:
                y[g] += out[q]
                count[g] += 1.0
    return s * y / count
