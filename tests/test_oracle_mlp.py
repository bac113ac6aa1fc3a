"""Pins of the fp64 policy-network oracle: central finite differences and
torch autograd (CPU, float64)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mlp


def _data(n=37, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, mlp.IN))
    t = np.stack([rng.integers(0, 2, n), rng.integers(0, 2, n),
                  rng.uniform(2, 7, n), rng.uniform(7, 11, n)], 1).astype(float)
    mask = (rng.random((n, 4)) < 0.8).astype(float)
    return x, t, mask


def test_param_count():
    assert mlp.NPARAMS == 1476


def test_grad_finite_differences():
    p = mlp.init_params(3)
    x, t, mask = _data()
    g = mlp.grad(p, x, t, mask)
    rng = np.random.default_rng(0)
    idx = rng.choice(mlp.NPARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, x, t, mask) - mlp.loss(p - e, x, t, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_grad_matches_autograd():
    torch = pytest.importorskip("torch")
    p = mlp.init_params(5)
    x, t, mask = _data(50, 2)
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(p).items()}
    X = torch.tensor(x)
    h1 = torch.relu(X @ P["W1"].T + P["b1"])
    h2 = torch.relu(h1 @ P["W2"].T + P["b2"])
    y = h2 @ P["W3"].T + P["b3"]
    T, M = torch.tensor(t), torch.tensor(mask)
    bce = torch.nn.functional.binary_cross_entropy_with_logits
    per = (M[:, 0] * bce(y[:, 0], T[:, 0], reduction="none") + M[:, 1] * bce(y[:, 1], T[:, 1], reduction="none")
           + M[:, 2] * 0.5 * (y[:, 2] - T[:, 2]) ** 2 + M[:, 3] * 0.5 * (y[:, 3] - T[:, 3]) ** 2)
    L = per.mean()
    L.backward()
    ref = np.concatenate([P[name].grad.numpy().ravel() for name, _ in mlp.SHAPES])
    np.testing.assert_allclose(mlp.grad(p, x, t, mask), ref, rtol=1e-10, atol=1e-14)
    assert abs(L.item() - mlp.loss(p, x, t, mask)) < 1e-12


def test_adam_reduces_loss():
    p = mlp.init_params(7)
    x, t, mask = _data(200, 3)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.loss(p, x, t, mask)
    for s in range(1, 201):
        p, m, v = mlp.adam(p, mlp.grad(p, x, t, mask), m, v, s, lr=3e-3)
    assert mlp.loss(p, x, t, mask) < 0.7 * l0
