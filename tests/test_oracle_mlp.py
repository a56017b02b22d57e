"""Oracle MLP of the learned coarse correction: backward checked by central
finite differences, GELU against its closed form values, Adam against a
hand-computed first step."""
import numpy as np
import pytest

from oracle import mlp


def test_gelu_values():
    # GELU(0) = 0, GELU(x) - GELU(-x) = x, GELU'(0) = 1/2
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    x = np.linspace(-3, 3, 13)
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-15)
    assert abs(mlp.gelu_prime(np.array([0.0]))[0] - 0.5) < 1e-15
    h = 1e-6
    assert np.allclose(mlp.gelu_prime(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-8)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(3) * 0.5 + 0.01 * rng.standard_normal(mlp.n_params())
    X = rng.standard_normal((7, 30))
    T = rng.standard_normal((7, 27))
    _, g = mlp.loss_and_grad(theta, X, T)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp.loss(theta + e, X, T) - mlp.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_first_step_is_signed_lr():
    opt = mlp.Adam(3, lr=0.01)
    theta = np.zeros(3)
    g = np.array([2.0, -0.5, 0.0])
    new = opt.step(theta, g)
    # first step: m_hat = g, v_hat = g^2  ->  -lr * sign(g) (0 for g = 0)
    assert np.allclose(new, -0.01 * np.sign(g), atol=1e-9)


def test_training_reduces_loss_on_linear_target():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((256, 30))
    M = rng.standard_normal((30, 27)) * 0.2
    T = X @ M
    theta = mlp.init_params(0)
    opt = mlp.Adam(theta.size, lr=3e-3)
    l0 = mlp.loss(theta, X, T)
    for _ in range(200):
        _, g = mlp.loss_and_grad(theta, X, T)
        theta = opt.step(theta, g)
    assert mlp.loss(theta, X, T) < 0.1 * l0


# -- the learned coarse correction (network per coarse cell, node averaging) --
def _coarse_space(k=2):
    from oracle import octree
    from oracle.space import Space
    return Space(octree.Octree(4), k)


def _zero_net(nq):
    return np.zeros(mlp.n_params(mlp.sizes_for(nq + 3)))


def _slices(nq):
    """Offsets of W1, b1, W2, b2, W3, b3 in the flat parameter vector."""
    nin = nq + 3
    off, out = 0, {}
    for name, size in (("W1", nin * 64), ("b1", 64), ("W2", 64 * 64), ("b2", 64), ("W3", 64 * nq), ("b3", nq)):
        out[name] = slice(off, off + size)
        off += size
    return out


def _G(z):
    """GELU(GELU(z)) from its closed form z Phi(z), Phi by the error function."""
    from scipy.special import erf
    g = lambda t: 0.5 * t * (1.0 + erf(t / np.sqrt(2.0)))
    return g(g(z))


def test_coarse_correction_constant_output_is_s():
    """Bias-only network with output 1 at every node: every DoF is the mean
    of ones times s = ||b||, whatever the number of cells around it; a sum
    instead of the mean, or a missing s, fails."""
    S = _coarse_space()
    nq = 27
    theta = _zero_net(nq)
    theta[_slices(nq)["b3"]] = 1.0
    b = np.random.default_rng(0).standard_normal(S.n_dofs)
    y = mlp.coarse_correction(theta, S, b)
    assert np.allclose(y, np.linalg.norm(b), rtol=1e-14)
    assert np.all(mlp.coarse_correction(theta, S, np.zeros(S.n_dofs)) == 0.0)


def test_coarse_correction_vertex_share():
    """Output 1 at the local vertex (0,0,0) only: an interior mesh vertex is
    that corner of exactly one of its 8 cells, so it gets s/8; a vertex on a
    face of the coarse grid next to the Dirichlet boundary is not a DoF, the
    cell-interior DoFs get 0."""
    S = _coarse_space()
    nq = 27
    theta = _zero_net(nq)
    theta[_slices(nq)["b3"].start + 0] = 1.0
    b = np.ones(S.n_dofs)
    y = mlp.coarse_correction(theta, S, b) / np.linalg.norm(b)
    pts = S.dof_points()
    h = 0.25
    on_vertex = np.all(np.abs(pts / h - np.round(pts / h)) < 1e-12, axis=1)
    assert on_vertex.sum() == 27  # the 3^3 interior vertices of the 4^3 grid
    assert np.allclose(y[on_vertex], 1.0 / 8.0, rtol=1e-14)
    centre = np.all(np.abs(pts / h - np.floor(pts / h) - 0.5) < 1e-12, axis=1)
    assert centre.sum() == 64 and np.all(y[centre] == 0.0)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_coarse_correction_centre_inputs(d):
    """Input nq + d is centre coordinate d: one hidden path G(centre_d) to all
    outputs, so the DoF at a cell's centre (Q2 interior node) gets s G(its own
    coordinate d)."""
    S = _coarse_space()
    nq = 27
    sl = _slices(nq)
    theta = _zero_net(nq)
    theta[sl["W1"].start + (nq + d) * 64 + 0] = 1.0   # W1[nq + d, 0]
    theta[sl["W2"].start + 0 * 64 + 0] = 1.0          # W2[0, 0]
    theta[sl["W3"].start:sl["W3"].start + nq] = 1.0   # W3[0, :]
    b = np.random.default_rng(1).standard_normal(S.n_dofs)
    s = np.linalg.norm(b)
    y = mlp.coarse_correction(theta, S, b)
    pts = S.dof_points()
    centre = np.all(np.abs(pts / 0.25 - np.floor(pts / 0.25) - 0.5) < 1e-12, axis=1)
    assert np.allclose(y[centre], s * _G(pts[centre, d]), rtol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_coarse_correction_node_inputs(axis):
    """Input q = a + 3b + 9c is b at local node (a, b, c): reading the node
    one half-cell past the centre along `axis` (local index 2 on that axis,
    1 on the others) sends b(centre + h/2 e_axis)/s through G to the cell
    centre's DoF."""
    S = _coarse_space()
    nq = 27
    sl = _slices(nq)
    idx = [1, 1, 1]
    idx[axis] = 2
    q = idx[0] + 3 * idx[1] + 9 * idx[2]
    theta = _zero_net(nq)
    theta[sl["W1"].start + q * 64 + 0] = 1.0
    theta[sl["W2"].start + 0] = 1.0
    theta[sl["W3"].start:sl["W3"].start + nq] = 1.0
    pts = S.dof_points()
    f = lambda p: 1.0 + p[:, 0] + 2.0 * p[:, 1] ** 2 - 3.0 * p[:, 2] ** 3
    b = f(pts)
    s = np.linalg.norm(b)
    y = mlp.coarse_correction(theta, S, b)
    centre = np.all(np.abs(pts / 0.25 - np.floor(pts / 0.25) - 0.5) < 1e-12, axis=1)
    shifted = pts[centre].copy()
    shifted[:, axis] += 0.125
    want = s * _G(f(shifted) / s)
    # a face node on the Dirichlet boundary has value 0 as input
    on_bnd = (shifted[:, axis] > 1.0 - 1e-12)
    want[on_bnd] = s * _G(0.0)
    assert np.allclose(y[centre], want, rtol=1e-13)
