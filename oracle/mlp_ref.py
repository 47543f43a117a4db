"""FP64 reference of the learned block screener's network (numpy).

TEST INFRASTRUCTURE ONLY (the GPU kernels are checked against it).  The network maps the
16 features of a (shell pair, grid batch) block to a predicted log10 block magnitude:

    z1 = W1 x + b1,  h1 = silu(z1)        (64)
    z2 = W2 h1 + b2, h2 = silu(z2)        (64)
    y  = w3 . h2 + b3                     (1)
    silu(z) = z / (1 + e^{-z})

Loss: weighted squared error, under-prediction weighted by `under` (default 10):
    L = (1/N) sum_s c_s (y_s - t_s)^2,  c_s = under if y_s < t_s else 1.
Adam with bias correction for the update.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

SIZES = (16, 64, 64, 1)


def init_params(seed: int = 0) -> Dict[str, np.ndarray]:
    rng = np.random.default_rng(seed)
    p = {}
    fan = [(16, 64), (64, 64), (64, 1)]
    for k, (i, o) in enumerate(fan, 1):
        p["W%d" % k] = rng.normal(scale=np.sqrt(2.0 / i), size=(o, i))
        p["b%d" % k] = np.zeros(o)
    return p


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, X) -> Tuple[np.ndarray, dict]:
    z1 = X @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["W3"].T[:, 0] + p["b3"][0]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)


def loss(y, t, under: float = 10.0) -> float:
    c = np.where(y < t, under, 1.0)
    return float(np.mean(c * (y - t) ** 2))


def backward(p, cache, y, t, under: float = 10.0) -> Dict[str, np.ndarray]:
    n = len(y)
    c = np.where(y < t, under, 1.0)
    dy = 2.0 * c * (y - t) / n
    g = {}
    g["W3"] = (dy @ cache["h2"])[None, :]
    g["b3"] = np.array([dy.sum()])
    d2 = dy[:, None] * p["W3"][0][None, :] * dsilu(cache["z2"])
    g["W2"] = d2.T @ cache["h1"]
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * dsilu(cache["z1"])
    g["W1"] = d1.T @ cache["X"]
    g["b1"] = d1.sum(0)
    return g


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def flatten(p) -> np.ndarray:
    """Parameter order used by the GPU kernels: W1, b1, W2, b2, W3, b3 (row-major)."""
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])


def unflatten(v: np.ndarray) -> Dict[str, np.ndarray]:
    v = np.asarray(v, np.float64)
    o = 0
    p = {}
    for k, shape in [("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)), ("b3", (1,))]:
        n = int(np.prod(shape))
        p[k] = v[o:o + n].reshape(shape)
        o += n
    return p


NPARAM = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1
