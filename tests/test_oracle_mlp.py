"""Pins of the cost-model network oracle (oracle/mlp.py) against facts that do
not come from it: a hand-evaluated one-unit network, central finite
differences of the loss, and two properties of Adam (the first step moves
every parameter by the learning rate; the step is unchanged when gradients
are scaled)."""
import math

import numpy as np

import oracle.mlp as M


def test_one_unit_network_matches_hand_evaluation():
    # D = H = 1: out = W2 tanh(W1 tanh(W0 x + b0) + b1) + b2
    W0, b0, W1, b1, W2, b2 = 0.7, -0.2, 1.3, 0.1, -0.8, 0.25
    p = np.array([W0, b0, W1, b1, W2, b2])
    xs = [-1.5, 0.0, 0.4, 2.0]
    out, _, _ = M.forward(p, np.array(xs)[:, None], 1, 1)
    for x, o in zip(xs, out):
        ref = W2 * math.tanh(W1 * math.tanh(W0 * x + b0) + b1) + b2
        assert abs(o - ref) <= 1e-15
    y = np.array([0.1, -0.3, 0.2, 0.0])
    ref_loss = sum((o - t) ** 2 for o, t in zip(out, y)) / 4
    assert abs(M.loss(p, np.array(xs)[:, None], y, 1, 1) - ref_loss) <= 1e-15


def test_gradient_matches_central_differences():
    D, H, N = 4, 6, 30
    rng = np.random.default_rng(2)
    X = rng.standard_normal((N, D))
    y = rng.standard_normal(N)
    p = rng.standard_normal(H * D + H + H * H + H + H + 1) * 0.5
    g = M.gradient(p, X, y, D, H)
    for k in range(p.size):
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += e
        pm[k] -= e
        fd = (M.loss(pp, X, y, D, H) - M.loss(pm, X, y, D, H)) / (2 * e)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)), k


def test_first_adam_step_moves_each_parameter_by_the_learning_rate():
    # with zero initial moments the bias-corrected first step is lr * g/|g|
    # (up to eps), whatever the gradient's size
    rng = np.random.default_rng(3)
    g = rng.standard_normal(50) * np.logspace(-3, 3, 50)
    p = rng.standard_normal(50)
    p1, _, _ = M.adam_update(p, g, np.zeros(50), np.zeros(50), 1, 0.01)
    step = p - p1
    assert np.allclose(np.abs(step), 0.01, rtol=1e-4)
    assert np.all(np.sign(step) == np.sign(g))


def test_adam_step_is_invariant_to_gradient_scale():
    rng = np.random.default_rng(4)
    p = rng.standard_normal(20)
    m, v = np.zeros(20), np.zeros(20)
    m2, v2 = np.zeros(20), np.zeros(20)
    q = p.copy()
    c = 1000.0
    for t in range(1, 8):
        g = rng.standard_normal(20)
        p, m, v = M.adam_update(p, g, m, v, t, 1e-3)
        q, m2, v2 = M.adam_update(q, c * g, m2, v2, t, 1e-3)
    # only eps (1e-8, added to sqrt(v)) breaks the invariance: each step
    # differs by at most about lr * eps / sqrt(v), so 7 steps stay well under 1e-7
    assert np.abs(p - q).max() <= 1e-7


def test_adam_training_reduces_the_loss():
    D, H, N = 3, 8, 60
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (N, D))
    y = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]
    p0 = rng.standard_normal(H * D + H + H * H + H + H + 1) * 0.3
    l0 = M.loss(p0, X, y, D, H)
    _, l1 = M.adam_train(p0, X, y, D, H, 1500, 1e-2)
    assert l1 < 0.1 * l0
