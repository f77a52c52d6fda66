"""Oracle for the schedule cost model: a float64 numpy MLP.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Not from the paper: the
cost model is a small fully connected network, Linear layers with ReLU
between them and a linear output, trained with masked mean-squared error on
log-times and the Adam update.  Everything here is the textbook definition,
written out in float64 with the analytic backward pass:

  forward   Z_l = H_{l-1} W_l^T + b_l,  H_l = relu(Z_l)  (last layer: H_L = Z_L)
  loss      L = sum M (H_L - T)^2 / max(1, sum M)
  backward  dZ_L = 2 M (H_L - T) / max(1, sum M)
            dW_l = dZ_l^T H_{l-1},  db_l = sum_rows dZ_l,  dH_{l-1} = dZ_l W_l
            dZ_{l-1} = dH_{l-1} * [Z_{l-1} > 0]
  Adam      m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
            p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np


def forward(params, X):
    """params: list of (W, b) with W out x in.  Returns the list of layer
    outputs H_0 = X, H_1, ..., H_L (post-activation; last layer linear)."""
    H = [np.asarray(X, dtype=np.float64)]
    for l, (W, b) in enumerate(params):
        Z = H[-1] @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        H.append(np.maximum(Z, 0.0) if l + 1 < len(params) else Z)
    return H


def masked_mse(P, T, M):
    """Loss and dL/dP of the masked mean-squared error."""
    P, T, M = (np.asarray(a, dtype=np.float64) for a in (P, T, M))
    denom = max(1.0, float(M.sum()))
    d = P - T
    return float((M * d * d).sum() / denom), 2.0 * M * d / denom


def backward(params, H, dOut):
    """Gradients [(dW_l, db_l)] of the loss given dL/dH_L = dOut."""
    grads = [None] * len(params)
    dZ = np.asarray(dOut, dtype=np.float64)
    for l in range(len(params) - 1, -1, -1):
        W = np.asarray(params[l][0], np.float64)
        grads[l] = (dZ.T @ H[l], dZ.sum(axis=0))
        if l > 0:
            dH = dZ @ W
            dZ = dH * (H[l] > 0.0)
    return grads


def loss_and_grads(params, X, T, M):
    H = forward(params, X)
    L, dP = masked_mse(H[-1], T, M)
    return L, backward(params, H, dP)


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v
