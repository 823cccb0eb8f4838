"""FP64 CPU reference of the picker network (TEST INFRASTRUCTURE).

The network is y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 (4 -> 64 -> 64 ->
45) with the masked mean-squared-error loss
L = sum(mask (Y - T)^2) / sum(mask).  The gradient below is the textbook
backward pass (chain rule through each affine map and ReLU), written out in
numpy; tests pin it to central finite differences and then use it to check
the GPU kernels.  Parameters are packed in the order W1, b1, W2, b2, W3, b3
(row-major), the same order as the library's.
"""
from __future__ import annotations

import numpy as np

SIZES = (4, 64, 64, 45)


def count() -> int:
    i, h1, h2, o = SIZES
    return h1 * i + h1 + h2 * h1 + h2 + o * h2 + o


def unpack(p: np.ndarray):
    i, h1, h2, o = SIZES
    p = np.asarray(p, dtype=np.float64)
    off = 0

    def take(r, c=None):
        nonlocal off
        n = r * (c or 1)
        v = p[off:off + n]
        off += n
        return v.reshape(r, c) if c else v

    W1 = take(h1, i); b1 = take(h1)
    W2 = take(h2, h1); b2 = take(h2)
    W3 = take(o, h2); b3 = take(o)
    return W1, b1, W2, b2, W3, b3


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(p, X, T, mask):
    Y, _ = forward(p, X)
    m = np.asarray(mask, dtype=np.float64)
    cnt = m.sum()
    return float((m * (Y - T) ** 2).sum() / (cnt if cnt > 0 else 1.0))


def grad(p, X, T, mask):
    """Packed gradient of `loss` with respect to the parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    Y, (X, Z1, H1, Z2, H2) = forward(p, X)
    m = np.asarray(mask, dtype=np.float64)
    cnt = m.sum() if m.sum() > 0 else 1.0
    dY = 2.0 * m * (Y - np.asarray(T, dtype=np.float64)) / cnt
    gW3 = dY.T @ H2
    gb3 = dY.sum(axis=0)
    dH2 = (dY @ W3) * (Z2 > 0)
    gW2 = dH2.T @ H1
    gb2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2) * (Z1 > 0)
    gW1 = dH1.T @ X
    gb1 = dH1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma and Ba 2015, Algorithm 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
