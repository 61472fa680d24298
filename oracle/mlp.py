"""FP64 reference of the scheduler's cost model -- TEST INFRASTRUCTURE.

A multilayer perceptron with two hidden layers of 64 units:
    h1 = relu(x W1 + b1),  h2 = relu(h1 W2 + b2),  y = h2 w3 + b3
trained on the mean squared error  L = mean_i (y_i - t_i)^2  with Adam
(Kingma and Ba, "Adam: A Method for Stochastic Optimization", 2015):
    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2
    p <- p - lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps)   (step k)

Parameters live in one flat vector (the layout the engine uses):
    W1 [F][64] (row = input feature), b1 [64], W2 [64][64], b2 [64],
    w3 [64], b3 [1].
Gradients are written out by hand (back-propagation) and pinned against
central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64


def n_params(F: int) -> int:
    return F * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1


def unpack(p: np.ndarray, F: int):
    o = 0
    W1 = p[o:o + F * HIDDEN].reshape(F, HIDDEN); o += F * HIDDEN
    b1 = p[o:o + HIDDEN]; o += HIDDEN
    W2 = p[o:o + HIDDEN * HIDDEN].reshape(HIDDEN, HIDDEN); o += HIDDEN * HIDDEN
    b2 = p[o:o + HIDDEN]; o += HIDDEN
    w3 = p[o:o + HIDDEN]; o += HIDDEN
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, w3, b3


def forward(p: np.ndarray, X: np.ndarray) -> np.ndarray:
    X = np.asarray(X, np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(p, np.float64), X.shape[1])
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ w3 + b3[0]


def loss(p, X, t) -> float:
    y = forward(p, X)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(p: np.ndarray, X: np.ndarray, t: np.ndarray):
    """Loss and its gradient with respect to the flat parameter vector."""
    X = np.asarray(X, np.float64)
    t = np.asarray(t, np.float64)
    F = X.shape[1]
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(p, np.float64), F)
    B = X.shape[0]
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3[0]
    r = y - t
    L = float(np.mean(r ** 2))
    dy = 2.0 * r / B                     # dL/dy
    gw3 = h2.T @ dy
    gb3 = np.array([dy.sum()])
    dh2 = np.outer(dy, w3)
    dz2 = dh2 * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, gb3])
    return L, g


def adam_step(p, g, m, v, k, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (k = 1 for the first); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** k)
    vh = v / (1.0 - b2 ** k)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
