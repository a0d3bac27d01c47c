"""ORACLE (test infrastructure only): float64 reference of the route-selection MLP.

The route decision of Algorithm 2 (Section III-B) is a threshold on one
statistic of the degree distribution.  The learned alternative is a
multilayer perceptron 66 -> 64 -> 64 -> 3 with ReLU hidden layers: inputs are
the 64-bin log-degree histogram divided by n plus log2 n and log2 m; outputs
are one logit per route (BFS then SV; SV; SV with the bounded-shortcut
policy).  Training minimises the mean softmax cross-entropy with plain SGD.

Weights are row-major [out, in]; x is [batch, in].
"""
from __future__ import annotations

import numpy as np

SIZES = (66, 64, 64, 3)


def init_params(seed: int = 0, dtype=np.float64):
    """He-uniform initial weights from a seeded numpy generator, zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for fin, fout in zip(SIZES[:-1], SIZES[1:]):
        lim = np.sqrt(6.0 / fin)
        params.append(rng.uniform(-lim, lim, size=(fout, fin)).astype(dtype))
        params.append(np.zeros(fout, dtype))
    return params


def forward(params, x):
    """Returns (logits, cache)."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    x = np.asarray(x, np.float64)
    a1 = x @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (x, a1, h1, a2, h2)


def loss_and_grads(params, x, y):
    """Mean cross-entropy over the batch and its gradients (same order as params)."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    z, (x, a1, h1, a2, h2) = forward(params, x)
    B = z.shape[0]
    zmax = z.max(axis=1, keepdims=True)
    ez = np.exp(z - zmax)
    p = ez / ez.sum(axis=1, keepdims=True)
    y = np.asarray(y, np.int64)
    loss = float(np.mean(-np.log(p[np.arange(B), y])))
    dz = p.copy()
    dz[np.arange(B), y] -= 1.0
    dz /= B
    gW3 = dz.T @ h2
    gb3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (a2 > 0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    gW1 = da1.T @ x
    gb1 = da1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def sgd_step(params, grads, lr: float):
    return [np.asarray(p, np.float64) - lr * g for p, g in zip(params, grads)]


def predict(params, x):
    z, _ = forward(params, x)
    return np.argmax(z, axis=1)
