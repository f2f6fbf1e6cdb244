"""Viewspace-gradient difference (Eq. 9) and gate initialisation (Eq. 10), FP64 (oracle; test only).

Eq. 9: d_t = (1/V) sum_v [dL_t^(v)/dp'_{t-1} - dL_{t-1}^(v)/dp'_{t-1}] with MSE losses of the render of
A_{t-1} against the ground truth of frame t and of frame t-1.  Both gradients are taken at the same
render, and the adjoint is linear in the image gradient, so the difference equals one backward with
image gradient  dMSE_t/dI - dMSE_{t-1}/dI = 2 (I_{t-1} - I_t) / (3 H W).  The oracle computes both forms.

Eq. 10: p_i = |d_i| / (|d_i| + median_j |d_j|); the gate parameter then solves Eq. 8's p_i =
sigmoid(a_i - tau log(-gamma0/gamma1)), i.e. a_i = logit(p_i) + tau log(-gamma0/gamma1).
Readings: L2 norm of the 2-vector, lower median (element (N-1)//2 of the sorted norms), p clamped to
[1e-6, 1 - 1e-6] (0/0 gives 1e-6).
Pinned by invariants: a static video gives d = 0; the one-pass and two-pass forms agree; a_i is invariant
to a positive rescaling of d; |d_i| = median gives p = 1/2 exactly.
"""
from __future__ import annotations

import math

import numpy as np

P_CLAMP = 1e-6


def mse_grad(render: np.ndarray, gt: np.ndarray) -> np.ndarray:
    """Gradient of mean((render - gt)^2) over 3HW with respect to the render."""
    return 2.0 * (np.asarray(render, np.float64) - np.asarray(gt, np.float64)) / render.size


def dt_image_gradient(gt_prev: np.ndarray, gt_cur: np.ndarray) -> np.ndarray:
    """Single-backward image gradient 2 (I_{t-1} - I_t) / (3HW)."""
    return 2.0 * (np.asarray(gt_prev, np.float64) - np.asarray(gt_cur, np.float64)) / gt_prev.size


def gate_init(d: np.ndarray, gamma0: float, gamma1: float, tau: float):
    """d [N,2] -> (p [N], a [N])."""
    nrm = np.linalg.norm(np.asarray(d, np.float64), axis=1)
    srt = np.sort(nrm)
    med = srt[(len(srt) - 1) // 2] if len(srt) else 0.0
    den = nrm + med
    with np.errstate(invalid="ignore", divide="ignore"):
        p = np.where(den > 0, nrm / np.where(den > 0, den, 1.0), 0.0)
    p = np.clip(p, P_CLAMP, 1.0 - P_CLAMP)
    a = np.log(p) - np.log1p(-p) + tau * math.log(-gamma0 / gamma1)
    return p, a
