"""Pins of the FP64 rank-predictor oracle (oracle/mlp.py): central finite
differences of the loss, a linear model trained to convergence against the
least-squares solution, and Adam steps computed by hand."""
import numpy as np

from oracle import mlp as M


def test_gradient_matches_central_differences():
    F, H = 5, 7
    rng = np.random.default_rng(3)
    theta = M.init_params(F, H, seed=1) + 0.1 * rng.standard_normal(M.n_params(F, H))
    X = rng.standard_normal((9, F))
    t = rng.standard_normal(9)
    g = M.grad(theta, X, t, F, H)
    h = 1e-6
    num = np.zeros_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        num[i] = (M.loss(theta + e, X, t, F, H) - M.loss(theta - e, X, t, F, H)) / (2 * h)
    assert np.max(np.abs(num - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_linear_model_converges_to_least_squares():
    """With identity activations the network is an affine map of X; full-batch
    gradient descent on the MSE reaches the least-squares fit."""
    F, H = 3, 4
    rng = np.random.default_rng(5)
    X = rng.standard_normal((40, F))
    t = X @ np.array([0.5, -1.0, 2.0]) + 0.3 + 0.01 * rng.standard_normal(40)
    A = np.hstack([X, np.ones((40, 1))])
    coef, *_ = np.linalg.lstsq(A, t, rcond=None)
    best = np.mean((A @ coef - t) ** 2)
    theta = M.init_params(F, H, seed=2)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    ident = lambda z: z
    for step in range(1, 6001):
        g = M.grad(theta, X, t, F, H, tanh=False)
        theta, m, v = M.adam_step(theta, g, m, v, step, 1e-2)
    final = M.loss(theta, X, t, F, H, act=ident)
    assert final <= best * (1 + 1e-6) + 1e-12
    # the composed affine map equals the least-squares coefficients
    W1, b1, W2, b2, W3, b3 = M.unpack(theta, F, H)
    w = (W3 @ W2 @ W1)[0]
    b = (W3 @ (W2 @ b1 + b2) + b3)[0]
    assert np.allclose(np.append(w, b), coef, atol=1e-5)


def test_adam_step_by_hand():
    theta = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    m = np.zeros(2)
    v = np.zeros(2)
    th1, m1, v1 = M.adam_step(theta, g, m, v, 1, 0.1)
    # first step: mhat = g, vhat = g^2, update = lr * sign(g) (up to eps)
    assert np.allclose(th1, theta - 0.1 * np.sign(g), atol=1e-7)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    g2 = np.array([-0.5, 0.25])
    th2, m2, v2 = M.adam_step(th1, g2, m1, v1, 2, 0.1)
    mh = (0.9 * m1 + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * v1 + 0.001 * g2 * g2) / (1 - 0.999 ** 2)
    assert np.allclose(th2, th1 - 0.1 * mh / (np.sqrt(vh) + 1e-8))


def test_layout_round_trip_and_count():
    F, H = 16, 64
    theta = np.arange(M.n_params(F, H), dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = M.unpack(theta, F, H)
    assert W1.shape == (64, 16) and W2.shape == (64, 64) and W3.shape == (1, 64)
    assert M.n_params(F, H) == 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1
    assert b3[0] == theta[-1] and W1[1, 0] == 16


def test_training_reduces_loss_on_a_smooth_target():
    F = 4
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (256, F))
    t = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    theta, losses = M.train(X, t, F, epochs=60, lr=3e-3, batch=64, seed=1)
    assert losses[-1] < 0.1 * np.var(t)
