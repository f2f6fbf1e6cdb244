"""Philox4x32-10 counter-based generator and the draws made from it (oracle; test only).

The generator is the one of Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC 2011): a 4 x 32-bit counter is mixed with a 2 x 32-bit key by ten rounds of two 32 x 32 -> 64-bit products
(multipliers 0xD2511F53 and 0xCD9E8D57) whose high and low halves are recombined with the other two words and
the round key, the key being bumped between rounds by the Weyl constants 0x9E3779B9 and 0xBB67AE85.  Written
here in plain numpy uint64 arithmetic; pinned by the published known-answer vectors.

Draws used by the method's stochastic parts (both sides compute the same integers from the same counters):
    uniform(x)   = ((x >> 9) + 1/2) / 2^23, in (0, 1) and exact in float32 (24 significant bits);
    gate noise   u of Gaussian i at step s: word 0 of Philox(ctr = (i, s, GATE_TAG, 0), key = seed);
    split normals of Gaussian i at densification round r: Box-Muller on the words of
                 Philox(ctr = (i, r, SPLIT_TAG, 0)) and Philox(ctr = (i, r, SPLIT_TAG, 1)).
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF
GATE_TAG = 0x67617465   # "gate"
SPLIT_TAG = 0x73706C74  # "splt"


def philox4x32_10(ctr, key):
    """ctr [..., 4], key [..., 2] (unsigned 32-bit values) -> [..., 4] uint32."""
    c = [np.asarray(ctr, np.uint64)[..., k] & MASK for k in range(4)]
    k0 = np.asarray(key, np.uint64)[..., 0] & MASK
    k1 = np.asarray(key, np.uint64)[..., 1] & MASK
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = c[0] * np.uint64(M0)
        p1 = c[2] * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, -1).astype(np.uint32)


def uniform(x):
    """uint32 -> float64 in (0, 1): the top 23 bits plus one half, scaled by 2^-23."""
    return ((np.asarray(x, np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) / float(1 << 23)


def split_seed(seed: int):
    return np.array([seed & MASK, (seed >> 32) & MASK], np.uint64)


def gate_uniforms(n: int, seed: int, step: int):
    """u [n] of the stochastic gate at optimiser step `step`."""
    i = np.arange(n, dtype=np.uint64)
    ctr = np.stack([i, np.full(n, step & MASK, np.uint64), np.full(n, GATE_TAG, np.uint64),
                    np.zeros(n, np.uint64)], -1)
    key = np.broadcast_to(split_seed(seed), (n, 2))
    return uniform(philox4x32_10(ctr, key)[:, 0])


def split_normals(idx, seed: int, rnd: int):
    """Six standard normals per Gaussian index in idx ([len(idx), 6], float64): Box-Muller on the four uniforms of
    each of two Philox blocks, (u0, u1) -> (r cos t, r sin t) and (u2, u3) likewise, r = sqrt(-2 ln u_even),
    t = 2 pi u_odd."""
    idx = np.asarray(idx, np.uint64)
    m = len(idx)
    out = []
    key = np.broadcast_to(split_seed(seed), (m, 2))
    for blk in range(2):
        ctr = np.stack([idx, np.full(m, rnd & MASK, np.uint64), np.full(m, SPLIT_TAG, np.uint64),
                        np.full(m, blk, np.uint64)], -1)
        u = uniform(philox4x32_10(ctr, key))
        for a, b in ((0, 1), (2, 3)):
            r = np.sqrt(-2.0 * np.log(u[:, a]))
            t = 2.0 * np.pi * u[:, b]
            out += [r * np.cos(t), r * np.sin(t)]
    return np.stack(out[:6], -1)
