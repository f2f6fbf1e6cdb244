"""Learned residual proposal: trains and evaluates the 24 -> 64 -> 64 -> 12 MLP of qg_proposal_* on the GPU.

The network predicts, per Gaussian and frame, the initial residual parameters that zero initialisation would
otherwise supply: pre-gate position residual l_p (3), gate logit a (1) and latents l_hat (8) (Sec. 3.2,
Eq. 5-8), from the Gaussian's recent reconstruction history and the Eq. 10 gate probability (see
qg_proposal_features).  Its forward and backward run in the library's BF16 matrix-core kernels and Adam
in qg_adam_multi; torch supplies device memory, the training-set statistics used for standardisation and
the random sample indices of each mini-batch.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import qg

N_IN, N_HID, N_OUT = 24, 64, 12
OFF = {"W1": (0, (64, 24)), "b1": (1536, (64,)), "W2": (1600, (64, 64)), "b2": (5696, (64,)),
       "W3": (5760, (12, 64)), "b3": (6528, (12,))}


def init_params(seed: int = 0) -> np.ndarray:
    """Uniform fan-in initialisation (bound sqrt(3 / fan_in) for the SiLU layers, sqrt(1 / fan_in) for the
    linear output), zero biases, from a fixed seed."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2412, 4469, 2000 + seed])))
    p = np.zeros(qg.PROPOSAL_PARAMS, np.float32)
    for name, fan_in, gain in (("W1", 24, 3.0), ("W2", 64, 3.0), ("W3", 64, 1.0)):
        off, shape = OFF[name]
        b = math.sqrt(gain / fan_in)
        p[off:off + int(np.prod(shape))] = rng.uniform(-b, b, size=int(np.prod(shape)))
    return p


def unpack(params) -> dict:
    p = np.asarray(params)
    return {k: p[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in OFF.items()}


class Proposal:
    def __init__(self, device="cuda", seed=0, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.device = torch.device(device)
        self.params = torch.as_tensor(init_params(seed), device=self.device)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.stats = torch.zeros(72, device=self.device)
        self.stats[24:48] = 1.0
        self.stats[60:72] = 1.0
        self.step_state = torch.zeros(4, dtype=torch.int32, device=self.device)
        self.loss = torch.zeros(1, device=self.device)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.segs = qg.adam_segments([self.params], [self.grad], [self.m], [self.v], [lr])
        self.ws_bytes = qg.qg_proposal_bwd_workspace_size()
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def set_stats(self, X: torch.Tensor, T: torch.Tensor, floor=1e-6):
        """Standardisation from a training set: X [24][S] features, T [12][S] targets."""
        xm, xs = X.double().mean(1), X.double().std(1).clamp_min(floor)
        tm, ts = T.double().mean(1), T.double().std(1).clamp_min(floor)
        self.stats.copy_(torch.cat([xm, 1.0 / xs, tm, ts]).float())

    def grad_step(self, X, T, idx=None, m=None, stream=None):
        """One Adam step on the samples idx (device uint32 columns of X/T), or on all columns."""
        S = X.shape[1]
        m = int(idx.numel()) if idx is not None else (S if m is None else m)
        qg.qg_proposal_bwd(m, idx, S, X.stride(0), X, T, self.params, self.stats, self.grad, self.loss, self.ws,
                           self.ws_bytes, stream)
        b1, b2 = self.betas
        qg.qg_adam_multi(self.segs, b1, b2, self.eps, 0, True, stream, step_state=self.step_state)

    def train(self, X, T, steps=400, batch=65536, seed=0, log_every=0, log=None):
        """Mini-batch Adam on (X [24][S], T [12][S]); returns the losses read every log_every steps."""
        S = X.shape[1]
        gen = torch.Generator(device=self.device)
        gen.manual_seed(seed)
        losses = []
        for k in range(steps):
            idx = torch.randint(0, S, (min(batch, S),), generator=gen, device=self.device, dtype=torch.int64)
            idx = idx.to(torch.int32)
            self.grad_step(X, T, idx)
            if log_every and (k % log_every == 0 or k == steps - 1):
                losses.append((k, float(self.loss.item())))
                if log:
                    log(f"proposal step {k}: loss {losses[-1][1]:.5f}")
        return losses

    def predict(self, X, out=None, stream=None):
        """[12][n] outputs for features X [24][n]."""
        n = X.shape[1]
        if out is None:
            out = torch.empty(12, n, device=self.device)
        qg.qg_proposal_fwd(n, X.stride(0), X, self.params, self.stats, out, out.stride(0), stream)
        return out


def features(A1, A2, A3, p, out=None, stream=None):
    """[24][n] proposal inputs from A_{t-1}, A_{t-2}, A_{t-3} ([59][n]) and the Eq. 10 probabilities p [n]."""
    n = A1.shape[1]
    if out is None:
        out = torch.empty(24, n, device=A1.device)
    qg.qg_proposal_features(n, A1.stride(0), A1, A2, A3, p, out, out.stride(0), stream)
    return out
