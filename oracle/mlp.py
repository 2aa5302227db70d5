"""CPU FP64 oracle of the warm-start network: a 3-layer perceptron f(x) = W3^T relu(W2^T relu(W1^T x + b1) + b2)
+ b3 applied row-wise, its mean-squared-error loss, the gradient by hand-written backpropagation and one Adam
step (Kingma & Ba 2015).  TEST INFRASTRUCTURE ONLY (see ``kot_oracle``).

Parameter layout (flat vector, row-major): W1 (F x H), b1 (H), W2 (H x H), b2 (H), W3 (H x 1), b3 (1).
"""
from __future__ import annotations

import numpy as np

__all__ = ["n_params", "unpack", "forward", "loss_and_grad", "adam_step"]


def n_params(F: int, H: int) -> int:
    return F * H + H + H * H + H + H + 1


def unpack(theta: np.ndarray, F: int, H: int):
    o = 0
    W1 = theta[o:o + F * H].reshape(F, H); o += F * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + H].reshape(H, 1); o += H
    b3 = theta[o:o + 1]; o += 1
    return W1, b1, W2, b2, W3, b3


def forward(theta, X, F, H):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64), F, H)
    Z1 = X @ W1 + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ W2 + b2
    A2 = np.maximum(Z2, 0.0)
    out = (A2 @ W3 + b3)[:, 0]
    return out, (X, Z1, A1, Z2, A2)


def loss_and_grad(theta, X, y, F, H):
    """loss = mean((f(x) - y)^2); gradient w.r.t. the flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(theta, F, H)
    out, (X, Z1, A1, Z2, A2) = forward(theta, X, F, H)
    N = X.shape[0]
    r = out - y
    loss = float(np.mean(r * r))
    dout = (2.0 / N) * r[:, None]            # N x 1
    gW3 = A2.T @ dout
    gb3 = dout.sum(axis=0)
    dA2 = dout @ W3.T
    dZ2 = dA2 * (Z2 > 0)
    gW2 = A1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dA1 = dZ2 @ W2.T
    dZ1 = dA1 * (Z1 > 0)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t >= 1 is the step count after this update)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
