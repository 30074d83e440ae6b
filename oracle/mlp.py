"""FP64 reference of the cost-model network -- TEST INFRASTRUCTURE ONLY.

The library learns the paper's group price C_i (a predicted execution time,
Sec. VI, Fig. 5) with a 3-layer perceptron F -> 64 -> 64 -> 1 with ReLU,
trained by mean squared error and Adam.  This module is the plain definition
in double precision, written from the textbook formulas (matrix products from
numpy), with no code shared with the GPU kernels:

  z1 = x W1^T + b1,  h1 = max(z1, 0)
  z2 = h1 W2^T + b2, h2 = max(z2, 0)
  y  = h2 W3^T + b3
  L  = mean((y - t)^2)

Backward by the chain rule; Adam with bias correction (Kingma & Ba, 2015).
Parameter layout (flat, row-major [out][in]): W1[64][F] b1[64] W2[64][64]
b2[64] W3[64] b3[1].
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64


def n_params(F: int) -> int:
    return HIDDEN * F + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1


def unpack(p, F: int):
    p = np.asarray(p, dtype=np.float64)
    i = 0
    W1 = p[i:i + HIDDEN * F].reshape(HIDDEN, F); i += HIDDEN * F
    b1 = p[i:i + HIDDEN]; i += HIDDEN
    W2 = p[i:i + HIDDEN * HIDDEN].reshape(HIDDEN, HIDDEN); i += HIDDEN * HIDDEN
    b2 = p[i:i + HIDDEN]; i += HIDDEN
    W3 = p[i:i + HIDDEN]; i += HIDDEN
    b3 = p[i]
    return W1, b1, W2, b2, W3, b3


def forward(p, x, F: int, keep=False):
    W1, b1, W2, b2, W3, b3 = unpack(p, F)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return (y, (x, z1, h1, z2, h2)) if keep else y


def loss(p, x, t, F: int) -> float:
    y = forward(p, x, F)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def loss_grad(p, x, t, F: int):
    """(L, dL/dp) by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F)
    y, (x, z1, h1, z2, h2) = forward(p, x, F, keep=True)
    n = x.shape[0]
    r = y - np.asarray(t, np.float64)
    L = float(np.mean(r * r))
    dy = 2.0 * r / n
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return L, g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init(F: int, seed: int):
    """He-style initial parameters (a training choice, not part of the model)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / F), (HIDDEN, F))
    W2 = rng.normal(0, np.sqrt(2.0 / HIDDEN), (HIDDEN, HIDDEN))
    W3 = rng.normal(0, np.sqrt(1.0 / HIDDEN), HIDDEN)
    return np.concatenate([W1.ravel(), np.zeros(HIDDEN), W2.ravel(), np.full(HIDDEN, 0.01), W3, [0.0]])
