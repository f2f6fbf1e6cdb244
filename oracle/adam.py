"""Adam update, FP64 (oracle; test only).

The paper optimises gates, residuals and decoders with Adam (App. B) without its moment constants; the
reading is beta = (0.9, 0.999), eps = 1e-8, bias-corrected:
    m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;  theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
Pinned against torch.optim.Adam in float64 (a library routine).
"""
from __future__ import annotations

import numpy as np


def adam_step(theta, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One step (t is the 1-based step count).  Returns new (theta, m, v)."""
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v
