"""Residual decode and position gate in torch FP64 (oracle; test only).

Eq. 4: A_t = A_{t-1} + R_t.  Eq. 5: l = STE(l_hat) (round to nearest in the forward pass, identity
gradient), r = D(l).  Sec. 3.2.2: position residual dp = g * l_p with the hard-concrete gate of Eq. 6-7
    g_hat = sigmoid(a / tau),  g_tilde = g_hat (gamma1 - gamma0) + gamma0,  g = min(1, max(0, g_tilde))
where a = log(alpha) is the learnable gate parameter, and the L0 surrogate of Eq. 8,
    L_reg = sum_i sigmoid(a_i - tau log(-gamma0 / gamma1)).
Readings (listed in the design notes):
    * rounding is round-half-to-even (torch.round);
    * the decoder is one shared bias-free two-layer MLP with SiLU, latent 8 -> hidden 32 -> 56 outputs
      (rotation 4, log-scale 3, opacity logit 1, SH 48), so zero latents decode to a zero residual;
    * residuals are added in the stored parameter space (mean, raw quaternion, log-scale, logit, SH);
    * L_reg is the mean over Gaussians (``reduction='sum'`` gives Eq. 8 literally);
    * the gate is deterministic as Eq. 6 is written (no noise sample).  A stochastic flag follows the hard
      concrete distribution Eq. 6 cites (Louizos et al.): g_hat = sigmoid((a + log u - log(1 - u)) / tau) with
      u ~ U(0, 1) drawn per Gaussian and step from the counter-based generator in philox.py; u = 1/2 gives
      the deterministic gate, and P(g > 0) = sigmoid(a - tau log(-gamma0 / gamma1)), Eq. 8's p_i.
Pinned by closed forms of the gate (values, zero/one thresholds, slope at a = 0 for both hyper-parameter
sets of the paper's gating table), zero-latent => zero-residual, spot values of the rounding, and
torch.nn.functional reference layers.
"""
from __future__ import annotations

import math

import torch


def ste_round(l_hat: torch.Tensor) -> torch.Tensor:
    return l_hat + (torch.round(l_hat) - l_hat).detach()


def mlp_decode(l: torch.Tensor, W1: torch.Tensor, W2: torch.Tensor) -> torch.Tensor:
    """r = W2 SiLU(W1 l) for l [N,L], W1 [H,L], W2 [M,H] -> [N,M]."""
    pre = l @ W1.T
    h = pre * torch.sigmoid(pre)
    return h @ W2.T


def logistic_noise(u) -> torch.Tensor:
    """log u - log(1 - u) of uniforms u in (0, 1) (a standard logistic sample)."""
    u = torch.as_tensor(u, dtype=torch.float64)
    return torch.log(u) - torch.log1p(-u)


def gate(a: torch.Tensor, gamma0: float, gamma1: float, tau: float, noise=None) -> torch.Tensor:
    """Eq. 6-7; noise (optional, [N]) is the logistic sample of the stochastic hard concrete gate."""
    g_hat = torch.sigmoid(a / tau) if noise is None else torch.sigmoid((a + noise) / tau)
    g_tilde = g_hat * (gamma1 - gamma0) + gamma0
    return torch.clamp(g_tilde, 0.0, 1.0)


def l_reg(a: torch.Tensor, gamma0: float, gamma1: float, tau: float, reduction: str = "mean") -> torch.Tensor:
    p = torch.sigmoid(a - tau * math.log(-gamma0 / gamma1))
    return p.mean() if reduction == "mean" else p.sum()


def decode(prev: torch.Tensor, latents: torch.Tensor, W1: torch.Tensor, W2: torch.Tensor, l_p: torch.Tensor,
           a: torch.Tensor, gamma0: float, gamma1: float, tau: float, noise=None):
    """prev [59,N] (planes), latents [L,N], W1 [H,L], W2 [56,H], l_p [3,N], a [N]; noise [N] optional (stochastic
    gate).

    Returns (attrs [59,N], g [N], L_reg mean)."""
    l = ste_round(latents.T)
    r = mlp_decode(l, W1, W2)  # [N,56]
    g = gate(a, gamma0, gamma1, tau, noise)
    dp = g[None, :] * l_p
    out = prev + torch.cat([dp, r.T], 0)
    return out, g, l_reg(a, gamma0, gamma1, tau)
