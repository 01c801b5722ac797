"""FP64 reference of the tile-selector network.

TEST INFRASTRUCTURE (part of the oracle): the GPU training kernels' forward
pass, gradients and Adam update are checked against these plain definitions.

Network: features (8) -> dense 64, ReLU -> dense 64, ReLU -> dense 12
(logits), trained with softmax cross-entropy against a target distribution
per sample, mean over the batch, and Adam (Kingma & Ba 2015, with bias
correction).

Parameter layout (packed, float32 on the GPU, 5,516 values):
    W1[8][64], b1[64], W2[64][64], b2[64], W3[64][12], b3[12]
row-major: W[i][o] multiplies input i into output o.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 8, 64, 12
SHAPES = [(N_IN, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_OUT), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)  # 5516


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])


def forward(p, X):
    """Hidden activations and logits: H1, H2, Z."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.maximum(X @ W1 + b1, 0.0)
    H2 = np.maximum(H1 @ W2 + b2, 0.0)
    Z = H2 @ W3 + b3
    return H1, H2, Z


def log_softmax(Z):
    Z = np.asarray(Z, dtype=np.float64)
    mx = Z.max(axis=1, keepdims=True)
    return Z - mx - np.log(np.exp(Z - mx).sum(axis=1, keepdims=True))


def loss(p, X, Q) -> float:
    """Mean over samples of -sum_c Q[n, c] log softmax(Z)[n, c]."""
    _, _, Z = forward(p, X)
    return float(-(np.asarray(Q) * log_softmax(Z)).sum(axis=1).mean())


def backward(p, X, Q) -> np.ndarray:
    """Gradient of `loss` by the chain rule, packed like the parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    H1, H2, Z = forward(p, X)
    P = np.exp(log_softmax(Z))
    dZ = (P - np.asarray(Q, dtype=np.float64)) / N
    gW3 = H2.T @ dZ
    gb3 = dZ.sum(axis=0)
    dH2 = (dZ @ W3.T) * (H2 > 0)
    gW2 = H1.T @ dH2
    gb2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2.T) * (H1 > 0)
    gW1 = X.T @ dH1
    gb1 = dH1.sum(axis=0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(p, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update at step t >= 1; returns (p, m, v)."""
    m = beta1 * np.asarray(m) + (1 - beta1) * np.asarray(g)
    v = beta2 * np.asarray(v) + (1 - beta2) * np.asarray(g) ** 2
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return np.asarray(p) - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / s[0]), size=s))
        else:
            parts.append(np.zeros(s))
    return pack(parts)
