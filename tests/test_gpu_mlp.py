"""GPU: the cost-model network's HIP forward / backward / Adam kernels against
a plain numpy FP64 reference and central finite differences."""
import numpy as np
import pytest

from paper_1709_02125_amd import ooc
import oracle.mlp as mlp_ref
from gpu_util import say

pytestmark = pytest.mark.gpu


def test_mlp_forward_and_gradient_match_reference():
    D, H, N = 12, 32, 80
    say("case: mlp gradient check")
    rng = np.random.default_rng(3)
    X = rng.standard_normal((N, D))
    y = rng.standard_normal(N)
    m = ooc.Mlp(D, H, seed=7)
    p = m.params()
    out_ref, _, _ = mlp_ref.forward(p, X, D, H)
    out = m.predict(X)
    assert np.abs(out - out_ref).max() <= 1e-12 * np.abs(out_ref).max()
    g, L = m.gradient(X, y)
    g_ref = mlp_ref.gradient(p, X, y, D, H)
    assert abs(L - mlp_ref.loss(p, X, y, D, H)) <= 1e-12 * L
    assert np.abs(g - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    # central differences on a spread of parameters
    for k in np.linspace(0, p.size - 1, 25).astype(int):
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += e
        pm[k] -= e
        fd = (mlp_ref.loss(pp, X, y, D, H) - mlp_ref.loss(pm, X, y, D, H)) / (2 * e)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), k
    m.close()


def test_mlp_training_reduces_loss():
    D, H, N = 6, 32, 120
    say("case: mlp training")
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (N, D))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - X[:, 3] ** 2
    m = ooc.Mlp(D, H, seed=11)
    _, l0 = m.gradient(X, y)
    l1 = m.train(X, y, epochs=2000, lr=3e-3)
    assert l1 < 0.05 * l0, (l0, l1)
    m.close()


def test_mlp_adam_training_matches_oracle():
    # the device's full-batch Adam epochs against the oracle's, from the same
    # starting parameters
    D, H, N = 12, 32, 64
    say("case: mlp adam vs oracle")
    rng = np.random.default_rng(5)
    X = rng.standard_normal((N, D))
    y = rng.standard_normal(N)
    m = ooc.Mlp(D, H, seed=13)
    p0 = m.params()
    l_dev = m.train(X, y, epochs=50, lr=1e-3)
    p_dev = m.params()
    p_ref, l_ref = mlp_ref.adam_train(p0, X, y, D, H, 50, 1e-3)
    assert np.abs(p_dev - p_ref).max() <= 1e-9 * np.abs(p_ref).max()
    assert abs(l_dev - l_ref) <= 1e-9 * l_ref
    m.close()
