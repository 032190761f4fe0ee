"""FP64 reference of the step-time cost model: a 2-hidden-layer ReLU MLP with MSE loss and Adam.

TEST INFRASTRUCTURE ONLY (checks the library's HIP training and inference kernels).

Parameter vector layout (shared with the library, row-major blocks in this order):
    W1 [H x F], b1 [H], W2 [H x H], b2 [H], w3 [H], b3 [1]
Inputs are standardised first: x' = (x - mean) / std.
    h1 = relu(W1 x' + b1);  h2 = relu(W2 h1 + b2);  y = w3 . h2 + b3
Loss over a batch of n samples: L = (1/n) sum (y_i - t_i)^2.
Adam (Kingma & Ba): m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def n_params(n_in: int, hidden: int) -> int:
    return hidden * n_in + hidden + hidden * hidden + hidden + hidden + 1


def unpack(theta, n_in: int, hidden: int):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + hidden * n_in].reshape(hidden, n_in); o += hidden * n_in
    b1 = theta[o:o + hidden]; o += hidden
    W2 = theta[o:o + hidden * hidden].reshape(hidden, hidden); o += hidden * hidden
    b2 = theta[o:o + hidden]; o += hidden
    w3 = theta[o:o + hidden]; o += hidden
    b3 = theta[o:o + 1]; o += 1
    assert o == theta.size
    return W1, b1, W2, b2, w3, b3


def forward(theta, X, n_in, hidden, mean=None, std=None):
    W1, b1, W2, b2, w3, b3 = unpack(theta, n_in, hidden)
    X = np.asarray(X, dtype=np.float64)
    if mean is not None:
        X = (X - np.asarray(mean, dtype=np.float64)) / np.asarray(std, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3[0]
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, t, n_in, hidden, mean=None, std=None) -> float:
    y, _ = forward(theta, X, n_in, hidden, mean, std)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def gradient(theta, X, t, n_in, hidden, mean=None, std=None):
    """dL/dtheta in the packed layout (backpropagation written out layer by layer)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, n_in, hidden)
    y, (Xs, z1, h1, z2, h2) = forward(theta, X, n_in, hidden, mean, std)
    n = y.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n
    gw3 = h2.T @ dy
    gb3 = np.array([dy.sum()])
    dz2 = np.outer(dy, w3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ Xs
    gb1 = dz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, gb3])


def adam(theta, grad, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; returns (theta, m, v). `step` counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Minibatch training with the shuffled order the library documents for
# tn_costmodel_train (the shuffle's random numbers cannot be passed in, so both
# sides implement the same counter-based generator from its published definition).
# ---------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 (Steele, Lea, Flood 2014) output for state x: add the golden-ratio
    increment, then the two xor-shift-multiply rounds and the final xor-shift."""
    x = (x + 0x9E3779B97F4A7C15) & _M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & _M64
    return x ^ (x >> 31)


def epoch_orders(n: int, epochs: int, seed: int):
    """The sample order of every epoch: Fisher-Yates (Durstenfeld) in place on the previous
    epoch's order (0..n-1 before the first), swap i with j = splitmix64(seed ^ splitmix64(
    e 2^32 + i)) mod (i + 1) for i = n-1 .. 1."""
    order = list(range(n))
    out = []
    for e in range(epochs):
        for i in range(n - 1, 0, -1):
            j = splitmix64((seed ^ splitmix64((e * (1 << 32) + i) & _M64)) & _M64) % (i + 1)
            order[i], order[j] = order[j], order[i]
        out.append(list(order))
    return out


def train(theta, X, t, n_in, hidden, mean, std, epochs: int, batch: int, lr: float, seed: int):
    """Minibatch Adam: per epoch, consecutive batches of `batch` samples of that epoch's order
    (the last one may be smaller), one gradient of the batch's mean squared error and one
    Adam update each.  Returns the parameters after training."""
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    step = 0
    for order in epoch_orders(X.shape[0], epochs, seed):
        for off in range(0, len(order), batch):
            idx = order[off:off + batch]
            g = gradient(theta, X[idx], t[idx], n_in, hidden, mean, std)
            step += 1
            theta, m, v = adam(theta, g, m, v, step, lr)
    return theta
