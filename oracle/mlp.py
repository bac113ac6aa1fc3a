"""FP64 reference of the per-iteration policy network — TEST INFRASTRUCTURE ONLY.

The network (a project extension, not in the paper): 8 frontier features ->
32 -> 32 -> 4, ReLU hidden layers, linear outputs.  Parameter vector layout
(1,476 floats): W1[32,8] row-major, b1[32], W2[32,32], b2[32], W3[4,32], b3[4].

Outputs: y0 = logit of "pull", y1 = logit of "ballot filter", y2 = log2 of
the small/medium bin threshold, y3 = log2 of the medium/large threshold.
Per-sample loss, with a non-negative weight (0/1 mask) per output:
    m0 * BCE(y0, t0) + m1 * BCE(y1, t1) + m2 * (y2 - t2)^2 / 2 + m3 * (y3 - t3)^2 / 2
(BCE on logits), averaged over the batch.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 8, 32, 4
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (OUT, HID)), ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(p, x):
    """x [N, 8] -> (y [N, 4], cache)."""
    P = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"].T + P["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t, mask):
    y, _ = forward(p, x)
    t = np.asarray(t, dtype=np.float64)
    mask = np.asarray(mask, dtype=np.float64)
    bce = lambda z, tt: np.maximum(z, 0) - z * tt + np.log1p(np.exp(-np.abs(z)))
    per = (mask[:, 0] * bce(y[:, 0], t[:, 0]) + mask[:, 1] * bce(y[:, 1], t[:, 1])
           + mask[:, 2] * 0.5 * (y[:, 2] - t[:, 2]) ** 2 + mask[:, 3] * 0.5 * (y[:, 3] - t[:, 3]) ** 2)
    return float(per.mean())


def grad(p, x, t, mask):
    """Gradient of `loss` with respect to the packed parameters (backprop)."""
    P = unpack(p)
    y, (x, z1, h1, z2, h2) = forward(p, x)
    t = np.asarray(t, dtype=np.float64)
    mask = np.asarray(mask, dtype=np.float64)
    n = x.shape[0]
    sig = lambda z: 1.0 / (1.0 + np.exp(-z))
    dy = np.empty_like(y)
    dy[:, 0] = mask[:, 0] * (sig(y[:, 0]) - t[:, 0])
    dy[:, 1] = mask[:, 1] * (sig(y[:, 1]) - t[:, 1])
    dy[:, 2] = mask[:, 2] * (y[:, 2] - t[:, 2])
    dy[:, 3] = mask[:, 3] * (y[:, 3] - t[:, 3])
    dy /= n
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    d2 = (dy @ P["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ P["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return pack(g)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba); step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-uniform initial weights, zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[1])
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    return pack(d)
