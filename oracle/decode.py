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
      paper mode (linear_decode) is Eq. 5 as written: one linear decoder per category with the latent
      dimensions of the quantisation table;
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


# Paper mode (Eq. 5 as written, Sec. 3.2.1 and the quantisation table): one shared linear decoder per attribute
# category, r_c = D_c rint(l_c), with the table's latent dimensions (N3DV: rotation 6, scaling 8, opacity 3,
# colour base 8, colour frequencies 4; Immersive has 12 for the frequencies).  Output planes of each category
# in the 59-plane layout: rotation 3..6, scaling 7..9, opacity 10, colour base (SH degree 0) 11..13, colour
# frequencies (higher SH) 14..58.
PAPER_CATEGORIES = (("rotation", 3, 4), ("scaling", 7, 3), ("opacity", 10, 1), ("color_base", 11, 3),
                    ("color_freq", 14, 45))
PAPER_DIMS_N3DV = (6, 8, 3, 8, 4)
PAPER_DIMS_IMMERSIVE = (6, 8, 3, 8, 12)


def linear_decode(latents: torch.Tensor, Ds, dims=PAPER_DIMS_N3DV) -> torch.Tensor:
    """Residual planes [56, N] (planes 3..58) of latents [sum(dims), N] through the per-category decoders
    Ds = [D_c [M_c, L_c]] (straight-through rounding of the latents)."""
    l = ste_round(latents)
    out, k = [], 0
    for (name, plane, M), L, D in zip(PAPER_CATEGORIES, dims, Ds):
        assert tuple(D.shape) == (M, L), (name, tuple(D.shape))
        out.append(D @ l[k:k + L])
        k += L
    return torch.cat(out, 0)


def decode_linear(prev: torch.Tensor, latents: torch.Tensor, Ds, l_p: torch.Tensor, a: torch.Tensor,
                  gamma0: float, gamma1: float, tau: float, dims=PAPER_DIMS_N3DV, noise=None):
    """Paper-mode decode: as decode() with the per-category linear decoders.  Returns (attrs, g, L_reg mean)."""
    r = linear_decode(latents, Ds, dims)
    g = gate(a, gamma0, gamma1, tau, noise)
    out = prev + torch.cat([g[None, :] * l_p, r], 0)
    return out, g, l_reg(a, gamma0, gamma1, tau)


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
