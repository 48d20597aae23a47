"""float64 reference of the proposal network (32 -> 256 -> 1, ReLU, logistic
output) and of its training step (binary cross-entropy, Adam).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH: the GPU forward, backward
and Adam kernels are checked against these definitions (with the GPU's bf16
rounding of inputs and weights applied to the reference's inputs).

    z = X W1 + b1,  h = max(z, 0),  logit = h W2 + b2
    loss = mean over rows of  softplus(logit) - y * logit      (BCE with logits)
    dlogit = (sigmoid(logit) - y) / n
    dW2 = h^T dlogit,  db2 = sum dlogit,  dz = dlogit W2^T * [z > 0]
    dW1 = X^T dz,      db1 = sum over rows of dz
Adam (Kingma & Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

IN, HIDDEN = 32, 256


def bf16(a) -> np.ndarray:
    """Rounds to the nearest bfloat16 (ties to even) and returns float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(X, W1, b1, W2, b2, round_hidden=False):
    """round_hidden: the hidden activations are rounded to bf16 before the
    output layer, as the GPU network stores them (their gradient is then
    taken straight through the rounding)."""
    Z = X @ W1 + b1
    H = np.maximum(Z, 0.0)
    if round_hidden:
        H = bf16(H)
    return Z, H, H @ W2 + b2


def loss(X, y, W1, b1, W2, b2, round_hidden=False) -> float:
    _, _, logit = forward(X, W1, b1, W2, b2, round_hidden)
    return float(np.mean(np.logaddexp(0.0, logit) - y * logit))


def grads(X, y, W1, b1, W2, b2, round_hidden=False) -> dict:
    n = X.shape[0]
    Z, H, logit = forward(X, W1, b1, W2, b2, round_hidden)
    dlogit = (1.0 / (1.0 + np.exp(-logit)) - y) / n
    dZ = np.outer(dlogit, W2) * (Z > 0)
    return {"W1": X.T @ dZ, "b1": dZ.sum(axis=0), "W2": H.T @ dlogit, "b2": float(dlogit.sum())}


def adam(params: dict, g: dict, state: dict, lr: float, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(np.asarray(params[k], dtype=np.float64)))
        v = state.setdefault("v_" + k, np.zeros_like(np.asarray(params[k], dtype=np.float64)))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * np.square(g[k])
        step = lr * (m / (1 - beta1 ** t)) / (np.sqrt(v / (1 - beta2 ** t)) + eps)
        params[k] = params[k] - step
