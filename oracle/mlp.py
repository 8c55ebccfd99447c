"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

Plain numpy FP64 definition of the schedule cost-model network: D inputs ->
H tanh -> H tanh -> 1 linear, mean-squared-error loss, gradient by the chain
rule written out layer by layer, and full-batch Adam (Kingma and Ba, 2015:
first and second moment estimates with bias correction, beta1 = 0.9,
beta2 = 0.999, eps = 1e-8).  Parameter layout: W0[H][D], b0[H], W1[H][H],
b1[H], W2[H], b2."""
import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def unpack(p, D, H):
    o = 0
    W0 = p[o:o + H * D].reshape(H, D); o += H * D
    b0 = p[o:o + H]; o += H
    W1 = p[o:o + H * H].reshape(H, H); o += H * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H].reshape(1, H); o += H
    b2 = p[o:o + 1]
    return W0, b0, W1, b1, W2, b2


def forward(p, X, D, H):
    W0, b0, W1, b1, W2, b2 = unpack(p, D, H)
    A1 = np.tanh(X @ W0.T + b0)
    A2 = np.tanh(A1 @ W1.T + b1)
    return (A2 @ W2.T + b2)[:, 0], A1, A2


def loss(p, X, y, D, H):
    out, _, _ = forward(p, X, D, H)
    return np.mean((out - y) ** 2)


def gradient(p, X, y, D, H):
    W0, b0, W1, b1, W2, b2 = unpack(p, D, H)
    N = X.shape[0]
    out, A1, A2 = forward(p, X, D, H)
    dO = (2.0 * (out - y) / N)[:, None]
    gW2 = dO.T @ A2
    gb2 = dO.sum(0)
    dZ2 = (dO @ W2) * (1 - A2 ** 2)
    gW1 = dZ2.T @ A1
    gb1 = dZ2.sum(0)
    dZ1 = (dZ2 @ W1) * (1 - A1 ** 2)
    gW0 = dZ1.T @ X
    gb0 = dZ1.sum(0)
    return np.concatenate([gW0.ravel(), gb0, gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam_update(p, g, m, v, t, lr, b1=BETA1, b2=BETA2, eps=EPS):
    """One Adam step at step number t >= 1; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def adam_train(p, X, y, D, H, epochs, lr):
    """Full-batch Adam from zero moments; returns (parameters, final loss)."""
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, epochs + 1):
        p, m, v = adam_update(p, gradient(p, X, y, D, H), m, v, t, lr)
    return p, loss(p, X, y, D, H)
