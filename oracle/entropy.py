"""Storage of a frame's residuals (the compression back end after the fit; Sec. 3.2 quantised latents, Eq. 6-8
gated positions), FP64 / integer (oracle; test only).

Readings: a Gaussian's latent symbols are rint(l_hat) per dimension (the values the decoder reads), held as
int8 in [-128, 127]; they are entropy coded with one adaptive-free model per latent dimension (the frame's
symbol histogram of that dimension); the position residuals are stored for the Gaussians whose gate is
non-zero only, as (index, dx, dy, dz) records (COO); the decoder weights are stored once per frame.

The lower bound of the coded latents is the empirical entropy: sum over dimensions k and symbols s of
-c_ks log2(c_ks / n), in bits.
"""
from __future__ import annotations

import numpy as np


def latent_symbols(latents: np.ndarray) -> np.ndarray:
    """latents [L][N] (float) -> int symbols [N][L] = rint(l_hat) (round half to even, as the decoder)."""
    return np.rint(np.asarray(latents, np.float64)).astype(np.int64).T


def histograms(symbols: np.ndarray, lo: int = -128, nbins: int = 256):
    """symbols [N][L] -> (counts [L][nbins] of symbol - lo, number outside [lo, lo + nbins))."""
    s = np.asarray(symbols, np.int64)
    L = s.shape[1]
    h = np.zeros((L, nbins), np.int64)
    inside = (s >= lo) & (s < lo + nbins)
    for k in range(L):
        h[k] = np.bincount(s[inside[:, k], k] - lo, minlength=nbins)
    return h, int((~inside).sum())


def empirical_entropy_bits(hist: np.ndarray) -> float:
    """Sum over the models of -sum_s c_s log2(c_s / n)."""
    total = 0.0
    for row in np.asarray(hist, np.float64):
        n = row.sum()
        nz = row[row > 0]
        total += float(-(nz * np.log2(nz / n)).sum()) if n > 0 else 0.0
    return total


def coo_nonzero(gate: np.ndarray) -> np.ndarray:
    """Indices of the Gaussians whose gate is non-zero (their position residuals are stored)."""
    return np.nonzero(np.asarray(gate) != 0)[0]
