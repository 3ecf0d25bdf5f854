"""Schedule cost-model MLP in float64: forward, loss, backward, Adam.

No passage of the paper defines this: it is an extension. The paper's
``schedule(auto)`` policy (sec. 3.2 grammar) leaves the schedule to the
implementation; here a small MLP predicts log2(time) of a loop under a
candidate schedule. Definitions (textbook):

* layers 32 -> 64 -> 64 -> 1, ``z = x W^T + b``, ReLU between layers with
  derivative 0 at 0, linear output;
* loss = mean over the batch of ``(y - t)^2``;
* Adam (Kingma & Ba 2015) with bias correction:
  ``m = b1 m + (1-b1) g``, ``v = b2 v + (1-b2) g^2``,
  ``p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)``.

Parameters are a dict ``W1 (64,32) b1 (64) W2 (64,64) b2 (64) W3 (1,64) b3 (1)``.
"""
from __future__ import annotations

import numpy as np

DIMS = (32, 64, 64, 1)
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(P, X):
    X = np.asarray(X, np.float64)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"].T + P["b3"]
    return y[:, 0], (X, z1, h1, z2, h2)


def loss(P, X, t):
    y, _ = forward(P, X)
    d = y - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(P, X, t):
    """Gradients of ``loss`` with respect to every parameter (chain rule)."""
    y, (X, z1, h1, z2, h2) = forward(P, X)
    B = X.shape[0]
    dy = (2.0 / B) * (y - np.asarray(t, np.float64))          # (B,)
    g = {}
    g["W3"] = dy[None, :] @ h2                                 # (1,64)
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] * P["W3"]                                # (B,64)
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ P["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(P, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step ``t`` (1-based); returns new (P, m, v)."""
    P2, m2, v2 = {}, {}, {}
    for k in NAMES:
        m2[k] = b1 * m[k] + (1 - b1) * g[k]
        v2[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m2[k] / (1 - b1 ** t)
        vh = v2[k] / (1 - b2 ** t)
        P2[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P2, m2, v2


def zeros_like(P):
    return {k: np.zeros_like(np.asarray(P[k], np.float64)) for k in NAMES}
