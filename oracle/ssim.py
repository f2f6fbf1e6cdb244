"""D-SSIM term of the image loss (Eq. 3), FP64 (oracle; test only).

Eq. 3 mixes an L1 term and a D-SSIM term with a weight lambda that the paper does not state; 0.2, the value of
the 3D-GS method it builds on, is the reading taken here, and the term is optional in the fit.  SSIM
follows Wang et al. (2004) as 3D-GS uses it: per channel, local statistics under an 11 x 11 Gaussian window
with sigma 1.5 (normalised to sum 1), zero padding outside the image ("same" size), C1 = 0.01^2,
C2 = 0.03^2 for a dynamic range of 1:
    mu_x = w * x, sigma_x^2 = w * x^2 - mu_x^2, sigma_xy = w * (x y) - mu_x mu_y,
    SSIM = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
and the loss term is D-SSIM = 1 - mean over pixels and channels of SSIM.  The convolution is a library
primitive (torch conv2d in float64); the gradient comes from autograd through these definitions.

Pinned by (tests/test_oracle_ssim.py): SSIM(x, x) = 1; symmetry in (x, y); the closed form for constant
images away from the border; the window's separability and normalisation; central finite differences.
"""
from __future__ import annotations

import math

import numpy as np
import torch

WIN = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window_1d(size: int = WIN, sigma: float = SIGMA) -> np.ndarray:
    """Normalised 1D Gaussian taps g[k] ~ exp(-(k - size//2)^2 / (2 sigma^2))."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def window_2d(size: int = WIN, sigma: float = SIGMA) -> np.ndarray:
    g = window_1d(size, sigma)
    return np.outer(g, g)


def _blur(t: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """t [C,H,W] -> per-channel 2D correlation with w (symmetric), zero padding, same size."""
    c = t.shape[0]
    k = w.shape[0]
    return torch.nn.functional.conv2d(t[None], w[None, None].expand(c, 1, k, k), padding=k // 2, groups=c)[0]


def ssim_map(x, y) -> torch.Tensor:
    """x, y [C,H,W] (float64 tensors or arrays) -> SSIM per pixel and channel [C,H,W]."""
    x = torch.as_tensor(x, dtype=torch.float64)
    y = torch.as_tensor(y, dtype=torch.float64)
    w = torch.as_tensor(window_2d())
    mx, my = _blur(x, w), _blur(y, w)
    sxx = _blur(x * x, w) - mx * mx
    syy = _blur(y * y, w) - my * my
    sxy = _blur(x * y, w) - mx * my
    num = (2.0 * mx * my + C1) * (2.0 * sxy + C2)
    den = (mx * mx + my * my + C1) * (sxx + syy + C2)
    return num / den


def dssim(render, gt, with_grad: bool = True):
    """D-SSIM = 1 - mean SSIM and, optionally, its gradient with respect to the render [C,H,W]."""
    x = torch.tensor(np.asarray(render, np.float64), requires_grad=with_grad)
    loss = 1.0 - ssim_map(x, np.asarray(gt, np.float64)).mean()
    if not with_grad:
        return float(loss.detach()), None
    loss.backward()
    return float(loss.detach()), x.grad.numpy()


def loss_eq3(render, gt, lam: float = 0.2):
    """(1 - lambda) L1 + lambda D-SSIM and its gradient (L1: mean over 3HW with sign(0) = 0)."""
    r = np.asarray(render, np.float64)
    g = np.asarray(gt, np.float64)
    d = r - g
    l1 = float(np.abs(d).mean())
    gl1 = np.sign(d) / d.size
    ds, gds = dssim(r, g)
    return (1.0 - lam) * l1 + lam * ds, (1.0 - lam) * gl1 + lam * gds
