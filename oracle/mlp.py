"""Float64 forward and backward pass of the (p, q) selector network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network: 16 inputs -> 64 (ReLU) -> 64 (ReLU) -> 40 logits, one logit per
point of the (p, q) grid.  Parameters are one flat vector theta in the order
    W1 (64 x 16, row-major: W1[o, i]), b1 (64),
    W2 (64 x 64), b2 (64),
    W3 (40 x 64), b3 (40)
(7848 values).  Rows of X are items.

Loss: binary cross-entropy with logits, averaged over the (item, output)
entries whose mask is 1:
    l(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)),
which equals -y log s(z) - (1 - y) log(1 - s(z)) with s the logistic
function, written in the form that does not overflow.

Update: Adam (Kingma and Ba, ICLR 2015) with bias correction.

Parity status: pinned (central finite differences of the loss, closed forms
at zero logits and for the first Adam step, fitting a tiny set).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 16, 64, 40
SHAPES = ((N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_OUT, N_HID), (N_OUT,))
N_PARAM = sum(int(np.prod(s)) for s in SHAPES)   # 7848


def unpack(theta: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def init(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases; float64."""
    g = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            b = np.sqrt(6.0 / s[1])
            parts.append(g.uniform(-b, b, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(theta: np.ndarray, X: np.ndarray):
    """Returns (H1, H2, Z): the two hidden activations (after ReLU) and the logits."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64))
    X = np.asarray(X, np.float64)
    H1 = np.maximum(X @ W1.T + b1, 0.0)
    H2 = np.maximum(H1 @ W2.T + b2, 0.0)
    Z = H2 @ W3.T + b3
    return H1, H2, Z


def bce_loss(Z: np.ndarray, Y: np.ndarray, M: np.ndarray) -> float:
    Z, Y, M = (np.asarray(a, np.float64) for a in (Z, Y, M))
    per = np.maximum(Z, 0.0) - Z * Y + np.log1p(np.exp(-np.abs(Z)))
    return float(np.sum(per * M) / max(np.sum(M), 1.0))


def backward(theta: np.ndarray, X: np.ndarray, H1: np.ndarray, H2: np.ndarray, Z: np.ndarray, Y: np.ndarray,
             M: np.ndarray) -> np.ndarray:
    """Gradient of bce_loss(forward(theta, X)[2], Y, M) with respect to theta (flat, same layout)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64))
    X = np.asarray(X, np.float64)
    cnt = max(float(np.sum(M)), 1.0)
    dZ = (1.0 / (1.0 + np.exp(-Z)) - Y) * M / cnt          # d loss / d z
    gW3 = dZ.T @ H2
    gb3 = dZ.sum(0)
    dH2 = (dZ @ W3) * (H2 > 0)
    gW2 = dH2.T @ H1
    gb2 = dH2.sum(0)
    dH1 = (dH2 @ W2) * (H1 > 0)
    gW1 = dH1.T @ X
    gb1 = dH1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(theta, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
