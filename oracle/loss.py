"""L1 reconstruction loss and PSNR, FP64 (oracle; test only).

Eq. 3 combines D-SSIM and L1 with a weight lambda the paper does not give; the fitted loss here is the
L1 term (mean over 3HW) plus lambda_reg L_reg (Eq. 11).  PSNR = 10 log10(1 / MSE) of the render clamped
to [0, 1] against the ground truth (the paper reports PSNR, Sec. 4.1).
Pinned by closed forms: L1(I, I) = 0, gradient sign(x)/(3HW) with sign(0) = 0, PSNR at MSE 1e-4 is 40 dB.
"""
from __future__ import annotations

import numpy as np


def l1(render, gt):
    r = np.asarray(render, np.float64)
    g = np.asarray(gt, np.float64)
    diff = r - g
    return float(np.abs(diff).mean()), np.sign(diff) / diff.size


def psnr(render, gt):
    r = np.clip(np.asarray(render, np.float64), 0.0, 1.0)
    mse = float(((r - np.asarray(gt, np.float64)) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)
