"""fp64 reference of the branching network - TEST INFRASTRUCTURE ONLY.

The network maps 5 features of a candidate variable to a prediction of
log2(1 + size of the subtree below branching on it): 64 hidden ReLU units,
one linear output.  The GPU evaluates it with bf16 weights and activations
and fp32 accumulation; this reference takes the same bf16-rounded weights
and inputs and computes everything else in fp64.

theta layout (449 values): W1[64][5] (row = hidden unit), b1[64], w2[64], b2.
"""
from __future__ import annotations

import numpy as np

F, H = 5, 64
NP = H * F + H + H + 1
OFF_W1, OFF_B1, OFF_W2, OFF_B2 = 0, H * F, H * F + H, H * F + 2 * H


def bf16_bits(x) -> np.ndarray:
    """fp32 -> bf16 bit patterns, round to nearest even (finite inputs)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def bf16_round(x) -> np.ndarray:
    return bf16_value(bf16_bits(x))


def unpack(theta):
    th = np.asarray(theta, dtype=np.float64)
    W1 = th[OFF_W1:OFF_B1].reshape(H, F)
    return W1, th[OFF_B1:OFF_W2], th[OFF_W2:OFF_B2], th[OFF_B2]


def forward(theta, X, quantized: bool = True):
    """y[s] for inputs X [N][5].  quantized: the GPU's arithmetic (bf16
    weights and hidden activations); else the exact real-valued network."""
    W1, b1, w2, b2 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    if quantized:
        W1 = bf16_round(W1)
        w2 = bf16_round(w2)
        X = bf16_round(X)
        b1 = np.asarray(b1, np.float32).astype(np.float64)
        b2 = float(np.float32(b2))
    pre = X @ W1.T + b1
    Hact = np.maximum(pre, 0.0)
    if quantized:
        Hact = bf16_round(Hact)
    return Hact @ w2 + b2, pre, Hact


def loss(theta, X, T, quantized: bool = True) -> float:
    y, _, _ = forward(theta, X, quantized)
    return float(np.mean((y - np.asarray(T, np.float64)) ** 2))


def grad(theta, X, T, quantized: bool = True):
    """d loss / d theta by backpropagation.  With quantized=True the bf16
    rounding of weights, inputs and activations counts as the identity
    (straight-through), as on the GPU."""
    W1, b1, w2, b2 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    if quantized:
        w2 = bf16_round(w2)
        X = bf16_round(X)
    y, pre, Hact = forward(theta, X, quantized)
    N = X.shape[0]
    dy = 2.0 * (y - np.asarray(T, np.float64)) / N
    g = np.zeros(NP)
    g[OFF_W2:OFF_B2] = Hact.T @ dy
    g[OFF_B2] = dy.sum()
    dpre = np.outer(dy, w2) * (pre > 0)
    g[OFF_W1:OFF_B1] = (dpre.T @ X).reshape(-1)
    g[OFF_B1:OFF_W2] = dpre.sum(axis=0)
    return g


def adam_step(theta, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma and Ba 2015), bias-corrected; returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_theta(seed: int = 0) -> np.ndarray:
    """He-style initial parameters (for training from scratch)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NP, dtype=np.float32)
    th[OFF_W1:OFF_B1] = rng.normal(0, np.sqrt(2.0 / F), H * F)
    th[OFF_B1:OFF_W2] = 0.01
    th[OFF_W2:OFF_B2] = rng.normal(0, np.sqrt(1.0 / H), H)
    th[OFF_B2] = 0.0
    return th
