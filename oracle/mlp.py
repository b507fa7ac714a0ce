"""Plain double-precision CPU reference of the learned-guess network
(test infrastructure only; the GPU library shares none of this code).

The network: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 . w3 + b3,
with x of 3 features, 64 hidden units per layer, and the loss
L = sum_s (y_s - t_s)^2 / n. The parameter vector is the flat float array
W1 [3][64] (input-major), b1 [64], W2 [64][64] (input-major), b2 [64],
w3 [64], b3 [1] (4481 values), the layout the library's kernels use.
"""
from __future__ import annotations

import numpy as np

H = 64
SIZES = [("W1", (3, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(theta, X):
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(theta, X, T, n_total=None):
    """Loss sum_s (y_s - t_s)^2 / n_total and its gradient (backpropagation
    written out layer by layer)."""
    p = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    n_total = len(T) if n_total is None else n_total
    r = y - np.asarray(T, dtype=np.float64)
    loss = float(np.sum(r * r) / n_total)
    dy = 2.0 * r / n_total
    g = {"b3": np.array([dy.sum()]), "w3": h2.T @ dy}
    dz2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)
