"""FP64 oracle of the per-row output-size predictor (an 8-64-64-1 ReLU MLP).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper has no predictor; this network sizes the accumulators and the
output of the one-pass SpGEMM path.  Written from the textbook definitions:
a fully connected ReLU network, mean-squared-error loss, reverse-mode
gradients by the chain rule, and Adam (Kingma and Ba, 2015, Algorithm 1 with
bias-corrected moments).

Parameters live in one flat vector with this layout (the same layout the
device kernels use):

    W1[64][8]  b1[64]  W2[64][64]  b2[64]  W3[64]  b3[1]      (4801 values)

Row-major weights: hidden unit h of layer 1 is relu(sum_f W1[h][f] x[f] + b1[h]).
"""
from __future__ import annotations

import numpy as np

NF, H1, H2 = 8, 64, 64
SIZES = [("W1", (H1, NF)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)),
         ("W3", (H2,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(theta: np.ndarray, x: np.ndarray):
    """Returns (y, cache): y has shape (N,)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2)


def loss(theta: np.ndarray, x: np.ndarray, t: np.ndarray) -> float:
    """Mean squared error (1/N) sum (y_i - t_i)^2."""
    y, _ = forward(theta, x)
    d = y - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d))


def grad(theta: np.ndarray, x: np.ndarray, t: np.ndarray):
    """(loss, flat gradient) of the mean squared error."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    y, (x, z1, h1, z2, h2) = forward(theta, x)
    n = x.shape[0]
    d = y - np.asarray(t, dtype=np.float64)
    dy = 2.0 * d / n
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, p["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean(d * d)), pack(g)


def adam_step(theta, g, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at 1-based step ``step``; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v

