"""FP64 oracle of the skeleton-rank predictor: a 3-layer tanh perceptron
F -> H -> H -> 1 trained with mean squared error and Adam.

Test infrastructure only (see oracle/__init__.py).  This part is not in the
paper; it follows the predictor described for the GPU path: per-group
features, target log2(1 + k) where k is the group's skeleton count, hidden
width 64, tanh activations, a linear output, MSE loss, Adam (Kingma and Ba,
"Adam: A Method for Stochastic Optimization", Algorithm 1, with bias
correction).

Parameter vector layout (shared with the C ABI, which documents it too):
W1 (H x F, row-major), b1 (H), W2 (H x H), b2 (H), W3 (1 x H), b3 (1).

Pinned by: central finite differences of the loss (tests/test_oracle_mlp.py),
a one-layer identity-activation model trained to convergence equal to the
least-squares solution, and hand-computed Adam steps.
"""
from __future__ import annotations

import numpy as np


def n_params(F: int, H: int = 64) -> int:
    return H * F + H + H * H + H + H + 1


def unpack(theta: np.ndarray, F: int, H: int = 64):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + H * F].reshape(H, F); o += H * F
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + H].reshape(1, H); o += H
    b3 = theta[o:o + 1]; o += 1
    assert o == theta.size
    return W1, b1, W2, b2, W3, b3


def init_params(F: int, H: int = 64, seed: int = 0) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((H, F), (H, H), (1, H)):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def forward(theta, X, F: int, H: int = 64, act=np.tanh):
    """Returns (y, cache) for inputs X (B x F)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, F, H)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = act(z1)
    z2 = h1 @ W2.T + b2
    h2 = act(z2)
    y = (h2 @ W3.T + b3)[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, t, F: int, H: int = 64, act=np.tanh) -> float:
    y, _ = forward(theta, X, F, H, act)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(theta, X, t, F: int, H: int = 64, tanh: bool = True):
    """Gradient of the MSE loss by the chain rule, layer by layer."""
    act = np.tanh if tanh else (lambda z: z)
    W1, b1, W2, b2, W3, b3 = unpack(theta, F, H)
    y, (X, z1, h1, z2, h2) = forward(theta, X, F, H, act)
    B = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / B          # dL/dy
    gW3 = dy[None, :] @ h2                                          # 1 x H
    gb3 = np.array([dy.sum()])
    dh2 = dy[:, None] * W3                                          # B x H
    dz2 = dh2 * (1.0 - h2 ** 2) if tanh else dh2
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (1.0 - h1 ** 2) if tanh else dh1
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(theta, g, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(X, t, F: int, H: int = 64, epochs: int = 200, lr: float = 1e-3, batch: int = 1024,
          seed: int = 0, theta=None):
    """Minibatch Adam in a fixed, seeded order; returns (theta, losses)."""
    rng = np.random.default_rng(seed)
    theta = init_params(F, H, seed) if theta is None else np.array(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    step = 0
    losses = []
    n = X.shape[0]
    for _ in range(epochs):
        order = rng.permutation(n)
        for s in range(0, n, batch):
            idx = order[s:s + batch]
            step += 1
            theta, m, v = adam_step(theta, grad(theta, X[idx], t[idx], F, H), m, v, step, lr)
        losses.append(loss(theta, X, t, F, H))
    return theta, losses
