"""Learned residual proposal: input features, the 24 -> 64 -> 64 -> 12 MLP and its backward, in NumPy FP64
(oracle; test only).

Not a method of the paper: a network that predicts each Gaussian's initial residual parameters of frame t
(pre-gate position residual l_p (3), gate logit a (1), latents l_hat (8); Sec. 3.2, Eq. 5-8) from its
history, standing in for zero initialisation.  The paper's analogue is the gate initialisation of Eq. 10.
Definitions taken here (listed in the design notes):

* features (24) of Gaussian i at frame t, from the reconstructions A_{t-1}, A_{t-2}, A_{t-3} (attribute
  planes 0..9: mean 3, quaternion 4, log-scale 3) and the Eq. 10 probability p_i of frame t:
      [ mean of A_{t-1} (3) | A_{t-1} - A_{t-2} on planes 0..9 (10) | A_{t-2} - A_{t-3} on planes 0..9 (10) | p_i ]
  (frames before the first use A_0, so the history starts at zero);
* standardisation: x_s = (x - in_mean) * in_rstd per feature; outputs y = y_s * out_std + out_mean;
* the network: h1 = SiLU(W1 x_s + b1), h2 = SiLU(W2 h1 + b2), y_s = W3 h2 + b3 (W1 [64][24],
  W2 [64][64], W3 [12][64]);
* BF16 operands with wider accumulation: every matrix operand (weights, x_s, h1, h2 and in the backward
  the output gradient, dL/d pre2 and dL/d pre1) is rounded to bfloat16 (from its float32 value, round to
  nearest even) before the product; biases, pre-activations and gradients' elementwise factors stay
  wide.  With ``rounding=False`` every operand stays FP64 (the plain MLP);
* training loss: L = (1/m) sum over the m samples and 12 outputs of (y_s - t_s)^2 with standardised
  targets t_s = (t - out_mean) / out_std.

Pinned by: the rounding against torch's float32 -> bfloat16 conversion (an independent implementation);
the unrounded forward against torch.nn.functional layers; every unrounded gradient against central finite
differences of the loss; the features on a hand-computed example.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 24, 64, 12


def bf16_round(x) -> np.ndarray:
    """float64 -> float32 (round to nearest) -> bfloat16 (round to nearest, ties to even), as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def _silu(x):
    return x / (1.0 + np.exp(-x))


def _silu_grad(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def features(A1, A2, A3, p) -> np.ndarray:
    """[24][n] features from A_{t-1}, A_{t-2}, A_{t-3} ([59][n] planes, only 0..9 are read) and p [n]."""
    A1, A2, A3 = (np.asarray(a, np.float64) for a in (A1, A2, A3))
    return np.concatenate([A1[0:3], A1[0:10] - A2[0:10], A2[0:10] - A3[0:10], np.asarray(p, np.float64)[None]])


def forward(x, W, stats, rounding=True):
    """x [24][m] raw features; W = dict(W1, b1, W2, b2, W3, b3); stats = dict(in_mean, in_rstd, out_mean,
    out_std).  Returns every intermediate (FP64)."""
    r = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(x, np.float64)
    xs = (x - stats["in_mean"][:, None]) * stats["in_rstd"][:, None]
    xb = r(xs)
    W1b, W2b, W3b = r(W["W1"]), r(W["W2"]), r(W["W3"])
    pre1 = W1b @ xb + np.asarray(W["b1"], np.float64)[:, None]
    h1b = r(_silu(pre1))
    pre2 = W2b @ h1b + np.asarray(W["b2"], np.float64)[:, None]
    h2b = r(_silu(pre2))
    ys = W3b @ h2b + np.asarray(W["b3"], np.float64)[:, None]
    y = ys * stats["out_std"][:, None] + stats["out_mean"][:, None]
    return dict(xb=xb, W1b=W1b, W2b=W2b, W3b=W3b, pre1=pre1, h1b=h1b, pre2=pre2, h2b=h2b, ys=ys, y=y)


def loss_and_grads(x, t, W, stats, rounding=True):
    """Training loss on m samples (x [24][m], raw targets t [12][m]) and its gradients with respect to
    W1, b1, W2, b2, W3, b3."""
    r = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    f = forward(x, W, stats, rounding)
    m = f["ys"].shape[1]
    ts = (np.asarray(t, np.float64) - stats["out_mean"][:, None]) / stats["out_std"][:, None]
    e = f["ys"] - ts
    loss = float((e * e).sum() / m)
    dy = 2.0 * e / m
    dyb = r(dy)
    dpre2 = (f["W3b"].T @ dyb) * _silu_grad(f["pre2"])
    dpre2b = r(dpre2)
    dpre1 = (f["W2b"].T @ dpre2b) * _silu_grad(f["pre1"])
    dpre1b = r(dpre1)
    g = dict(W3=dyb @ f["h2b"].T, b3=dy.sum(1), W2=dpre2b @ f["h1b"].T, b2=dpre2.sum(1),
             W1=dpre1b @ f["xb"].T, b1=dpre1.sum(1))
    return loss, g, f
