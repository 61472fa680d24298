"""Pins of the FP64 cost-model reference (oracle/mlp.py): the gradient
against central finite differences, Adam's first step against its closed
form, and training reduces the loss."""
import numpy as np

from oracle import mlp


def _data(seed, B=40, F=23):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(size=(B, F))
    t = rng.normal(size=B)
    p = rng.normal(scale=0.3, size=mlp.n_params(F))
    return X, t, p


def test_parameter_count():
    assert mlp.n_params(23) == 23 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def test_gradient_matches_central_differences():
    X, t, p = _data(1)
    L, g = mlp.grad(p, X, t)
    assert abs(L - mlp.loss(p, X, t)) < 1e-12
    rng = np.random.Generator(np.random.PCG64(2))
    idx = rng.choice(p.size, size=300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_matches_explicit_sums():
    X, t, p = _data(3, B=3, F=4)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p, 4)
    for i in range(3):
        h1 = [max(0.0, sum(X[i, f] * W1[f, j] for f in range(4)) + b1[j]) for j in range(64)]
        h2 = [max(0.0, sum(h1[a] * W2[a, j] for a in range(64)) + b2[j]) for j in range(64)]
        y = sum(h2[j] * w3[j] for j in range(64)) + b3[0]
        assert abs(y - mlp.forward(p, X)[i]) < 1e-9


def test_adam_first_step_closed_form():
    """After the first step m_hat = g and v_hat = g^2, so each parameter moves
    by lr * g / (|g| + eps): about lr against the sign of its gradient."""
    rng = np.random.Generator(np.random.PCG64(4))
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-3, 1e-8
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=lr, eps=eps)
    np.testing.assert_allclose(p - p1, lr * g / (np.abs(g) + eps), rtol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.Generator(np.random.PCG64(5))
    X = rng.normal(size=(256, 23))
    t = np.log1p(np.exp(X[:, :8]).sum(axis=1))  # a smooth target of the features
    p = rng.normal(scale=0.1, size=mlp.n_params(23))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss(p, X, t)
    for k in range(1, 301):
        _, g = mlp.grad(p, X, t)
        p, m, v = mlp.adam_step(p, g, m, v, k, lr=3e-3)
    assert mlp.loss(p, X, t) < 0.05 * L0
