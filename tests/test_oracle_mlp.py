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
