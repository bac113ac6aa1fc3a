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


def test_adam_first_step_closed_form():
    """Step 1 from zero moments: both bias corrections cancel the (1 - beta)
    factors, so the update is lr * g / (|g| + eps) element by element, whatever
    beta1 and beta2 are; m = (1 - beta1) g and v = (1 - beta2) g^2."""
    rng = np.random.default_rng(11)
    p = rng.normal(size=mlp.NPARAMS)
    g = rng.normal(size=mlp.NPARAMS) * np.exp(rng.uniform(-8, 2, mlp.NPARAMS))
    g[:5] = 0.0
    for lr, b1, b2, eps in [(1e-3, 0.9, 0.999, 1e-8), (0.05, 0.5, 0.75, 1e-3)]:
        p1, m1, v1 = mlp.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=lr, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(p - p1, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(m1, (1 - b1) * g, rtol=1e-15, atol=0)
        np.testing.assert_allclose(v1, (1 - b2) * g * g, rtol=1e-15, atol=0)


def test_adam_matches_torch_optim():
    """Several steps against torch.optim.Adam (float64, CPU) with a fresh
    gradient at every step: parameters and both moment estimates."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    p0 = rng.normal(size=mlp.NPARAMS)
    grads = [rng.normal(size=mlp.NPARAMS) * 10.0 ** rng.uniform(-6, 1) for _ in range(7)]
    for lr, b1, b2, eps in [(1e-3, 0.9, 0.999, 1e-8), (3e-2, 0.8, 0.95, 1e-6)]:
        w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([w], lr=lr, betas=(b1, b2), eps=eps)
        p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        for step, g in enumerate(grads, start=1):
            w.grad = torch.tensor(g, dtype=torch.float64)
            opt.step()
            p, m, v = mlp.adam(p, g, m, v, step, lr=lr, b1=b1, b2=b2, eps=eps)
            st = opt.state[w]
            # torch forms the moments with lerp / addcmul: the same values up
            # to rounding order, hence a few ulps of slack where terms cancel
            scale = np.abs(g).max()
            np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(m, st["exp_avg"].numpy(), rtol=1e-12, atol=1e-15 * scale)
            np.testing.assert_allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-15 * scale * scale)


def test_forward_single_layer_closed_forms():
    """Hand-computable networks: with W1 = I on the first 8 hidden units, W2 =
    I and W3 picking units, the outputs are ReLU(x) of chosen inputs plus the
    output bias; with every weight zero the output is b3 whatever x is."""
    d = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    d["W1"][:8, :8] = np.eye(8)
    d["W2"][:8, :8] = np.eye(8)
    d["W3"][0, 0] = 1.0
    d["W3"][1, 3] = -2.0
    d["W3"][2, 5] = 0.5
    d["b3"][:] = [0.25, -1.0, 3.0, 7.0]
    x = np.array([[1.5, -1, 0, 2, 0, -4, 0, 0], [-2, 0, 0, -1, 0, 3, 0, 0]], dtype=float)
    y, _ = mlp.forward(mlp.pack(d), x)
    expect = np.array([[1.5 + 0.25, -2 * 2 - 1.0, 0.5 * 0 + 3.0, 7.0],
                       [0 + 0.25, 0 - 1.0, 0.5 * 3 + 3.0, 7.0]])
    np.testing.assert_array_equal(y, expect)
    z = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    z["b3"][:] = [1, 2, 3, 4]
    y0, _ = mlp.forward(mlp.pack(z), np.random.default_rng(0).normal(size=(5, 8)))
    np.testing.assert_array_equal(y0, np.tile([1.0, 2, 3, 4], (5, 1)))
