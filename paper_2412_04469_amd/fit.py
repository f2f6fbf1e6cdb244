"""Per-frame residual fitting (Sec. 3.2-3.4, Eq. 4-11) driven entirely through the C ABI.

One optimiser iteration on one training view (one epoch covers all views, Sec. 4.1) enqueues:
    qg_decode_project -> qg_bin -> qg_render_fwd -> qg_l1_loss -> qg_render_decode_bwd -> qg_adam_multi
(or the unfused qg_decode_residuals -> qg_project -> ... -> qg_render_bwd -> qg_decode_residuals_bwd)
on the current stream with no host synchronisation.  The fitted quantities per frame are the
latents, the shared decoder weights, the pre-gate position residuals l_p and the gate logits a
(Eq. 5-8); A_{t-1} stays fixed (Eq. 4).  Loss: L1 + lambda_reg * L_reg (Eq. 3 without D-SSIM, Eq. 11).

Hyper-parameters (gating table and App. B of the paper, N3DV column by default): gate LR 0.1,
lambda_reg 0.01, gamma0 -0.5, gamma1 1.01, tau 0.3; position-residual LR 1.6e-4; decoder LR 1e-3;
Adam with beta = (0.9, 0.999), eps = 1e-8.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import qg
from .raster import Rasterizer


@dataclasses.dataclass
class FitConfig:
    gamma0: float = -0.5
    gamma1: float = 1.01
    tau: float = 0.3
    lambda_reg: float = 0.01
    lr_gate: float = 0.1
    lr_pos: float = 1.6e-4
    lr_latent: float = 0.01
    lr_decoder: float = 1e-3
    betas: tuple = (0.9, 0.999)
    eps: float = 1e-8
    latent_dim: int = 8
    hidden: int = 32
    tile: tuple = (16, 16)
    sh_degree: int = 3
    dilation: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)


def xavier_decoder(seed: int, L=8, H=32, M=56):
    """Xavier-uniform W1 [H][L], W2 [M][H] from a fixed seed (decoders need non-zero weights at frame 1)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2412, 4469, 1000 + seed])))
    a1 = math.sqrt(6.0 / (L + H))
    a2 = math.sqrt(6.0 / (H + M))
    return (rng.uniform(-a1, a1, size=(H, L)).astype(np.float32), rng.uniform(-a2, a2, size=(M, H)).astype(np.float32))


class FrameFitter:
    """Holds A_{t-1}, the residual parameters of frame t and their Adam state; all views share one resolution."""

    def __init__(self, prev_attrs: torch.Tensor, cams, gts, cfg: FitConfig = FitConfig(), W1=None, W2=None,
                 capacity=None, seed=0):
        self.cfg = cfg
        self.prev = prev_attrs.contiguous()
        self.n = int(self.prev.shape[1])
        self.ld = int(self.prev.stride(0))
        self.cams = list(cams)
        self.gts = gts
        dev = self.prev.device
        n, L, H = self.n, cfg.latent_dim, cfg.hidden
        if W1 is None:
            W1, W2 = xavier_decoder(seed, L, H, 56)
        self.W1 = torch.as_tensor(W1, device=dev).contiguous()
        self.W2 = torch.as_tensor(W2, device=dev).contiguous()
        self.lat = torch.zeros(L, n, device=dev)
        self.lp = torch.zeros(3, n, device=dev)
        self.a = torch.zeros(n, device=dev)
        self.params = {"lat": self.lat, "lp": self.lp, "a": self.a, "W1": self.W1, "W2": self.W2}
        self.lrs = {"lat": cfg.lr_latent, "lp": cfg.lr_pos, "a": cfg.lr_gate, "W1": cfg.lr_decoder,
                    "W2": cfg.lr_decoder}
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.t = 0
        self.attrs = torch.empty_like(self.prev)
        self.gate = torch.empty(max(n, 1), device=dev)
        self.lreg_part = torch.empty(qg.qg_decode_lreg_blocks(n), device=dev)
        self.grad_attrs = torch.zeros_like(self.prev)
        self.dws_bytes = qg.qg_decode_bwd_workspace_size(n, L, H, 56)
        self.dws = torch.empty(self.dws_bytes, dtype=torch.uint8, device=dev)
        self.fws_bytes = qg.qg_render_decode_bwd_workspace_size(n, 1)
        self.fws = torch.empty(self.fws_bytes, dtype=torch.uint8, device=dev)
        self.fused = True
        keys = list(self.params)
        self.adam_segs = qg.adam_segments([self.params[k] for k in keys], [self.grads[k] for k in keys],
                                          [self.m[k] for k in keys], [self.v[k] for k in keys],
                                          [self.lrs[k] for k in keys])
        self.rast = Rasterizer(n, [self.cams[0]], tile=cfg.tile, sh_degree=cfg.sh_degree, dilation=cfg.dilation,
                               bg=cfg.bg, device=dev, capacity=capacity)
        self.qcams = [qg.camera_array([c]) for c in self.cams]
        img = self.rast.images[0]
        self.count = img.numel()
        self.grad_img = torch.empty_like(img)
        self.loss_part = torch.empty(2 * qg.qg_loss_blocks(self.count), dtype=torch.float64, device=dev)
        self.loss_out = torch.zeros(2, dtype=torch.float64, device=dev)

    def reset_frame(self, prev_attrs=None, gts=None, a_init=None):
        """New frame: latents and position residuals restart at zero, decoder is warm-started, Adam resets."""
        if prev_attrs is not None:
            self.prev.copy_(prev_attrs)
        if gts is not None:
            self.gts = gts
        self.lat.zero_()
        self.lp.zero_()
        if a_init is None:
            self.a.zero_()
        else:
            self.a.copy_(a_init)
        for k in self.params:
            self.m[k].zero_()
            self.v[k].zero_()
            self.grads[k].zero_()
        self.t = 0

    # -- the step ------------------------------------------------------------------------------
    def decode(self, stream=None):
        c = self.cfg
        qg.qg_decode_residuals(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                               self.lp, self.a, c.gamma0, c.gamma1, c.tau, self.attrs, self.gate, self.lreg_part,
                               stream)

    def forward_view(self, v, stream=None):
        self.rast.qcams = self.qcams[v]
        self.rast.project(self.attrs, stream)
        self.rast.bin(stream)
        self.rast.render(stream)
        return self.rast.images[0]

    def step(self, v, stream=None):
        """One optimiser iteration on training view v (enqueue only)."""
        c = self.cfg
        r = self.rast
        if self.fused:
            r.qcams = self.qcams[v]
            qg.qg_decode_project(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                                 self.lp, self.a, c.gamma0, c.gamma1, c.tau, c.sh_degree, r.qcams, r.tile, c.dilation,
                                 r.t_proj, None, self.gate, None, stream)
            r.bin(stream)
            r.render(stream)
        else:
            self.decode(stream)
            self.forward_view(v, stream)
        qg.qg_l1_loss(self.count, r.images[0], self.gts[v], 1.0, self.grad_img, self.loss_part, stream)
        # parameter gradients are zero here: they start zeroed and qg_adam_multi clears them after use
        if self.fused:
            qg.qg_render_decode_bwd(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                                    self.lp, self.a, c.gamma0, c.gamma1, c.tau, c.lambda_reg, c.sh_degree, r.qcams,
                                    r.tile, c.dilation, r.t_proj, r.vals, r.ranges, r.bg, r.t_tf, r.t_last,
                                    [self.grad_img], self.grads["lat"], self.grads["W1"], self.grads["W2"],
                                    self.grads["lp"], self.grads["a"], None, None, self.fws, self.fws_bytes, stream)
        else:
            qg.qg_zero(self.grad_attrs, self.grad_attrs.numel() * 4, stream)
            r.backward(self.attrs, [self.grad_img], self.grad_attrs, stream=stream)
            qg.qg_decode_residuals_bwd(self.n, self.ld, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56, self.lp,
                                       self.a, c.gamma0, c.gamma1, c.tau, self.grad_attrs, c.lambda_reg,
                                       self.grads["lat"], self.grads["W1"], self.grads["W2"], self.grads["lp"],
                                       self.grads["a"], self.dws, self.dws_bytes, stream)
        self.t += 1
        b1, b2 = c.betas
        qg.qg_adam_multi(self.adam_segs, b1, b2, c.eps, self.t, True, stream)

    def loss_value(self, stream=None):
        """L1 of the last step (host sync)."""
        qg.qg_loss_reduce(self.count, self.loss_part, self.loss_out, stream)
        return float(self.loss_out[0].item())

    def psnr(self, cam, gt, stream=None):
        """PSNR of the decoded frame rendered at ``cam`` against ``gt`` (host sync)."""
        self.decode(stream)
        self.rast.qcams = qg.camera_array([cam])
        self.rast.project(self.attrs, stream)
        self.rast.bin(stream)
        if self.rast.ensure_capacity():
            self.rast.bin(stream)
        self.rast.render(stream)
        qg.qg_l1_loss(self.count, self.rast.images[0], gt, 1.0, None, self.loss_part, stream)
        qg.qg_loss_reduce(self.count, self.loss_part, self.loss_out, stream)
        mse = float(self.loss_out[1].item())
        return float("inf") if mse <= 0 else -10.0 * math.log10(mse)

    def size_capacity(self, margin=1.3):
        """Bin every view once (host syncs) and size the pair capacity for all of them."""
        worst = 0
        self.decode()
        for v in range(len(self.cams)):
            self.rast.qcams = self.qcams[v]
            self.rast.project(self.attrs)
            self.rast.bin()
            worst = max(worst, int(self.rast.num_pairs.item()))
        if worst * 1.05 > self.rast.capacity:
            self.rast._alloc_capacity(int(worst * margin))
        return worst


def render_views(attrs: torch.Tensor, cams, cfg: FitConfig = FitConfig(), capacity=None):
    """Forward renders of ``attrs`` at each camera (used to make ground-truth frames of synthetic scenes)."""
    out = []
    rast = Rasterizer(attrs.shape[1], [cams[0]], tile=cfg.tile, sh_degree=cfg.sh_degree, dilation=cfg.dilation,
                      bg=cfg.bg, device=attrs.device, capacity=capacity)
    for c in cams:
        rast.qcams = qg.camera_array([c])
        rast.forward(attrs)
        out.append(rast.images[0].clone())
    return out


def viewspace_gradient_difference(prev_attrs: torch.Tensor, cams, gt_prev, gt_cur, cfg: FitConfig = FitConfig(),
                                  capacity=None):
    """Sum over views of Eq. 9's bracket: d [2][n] (the 1/V factor of Eq. 9 is left out; Eq. 10 is scale-free).

    Each view: render A_{t-1}, then one adjoint pass with image gradient 2 (I_{t-1} - I_t) / (3HW), reading
    dL/dp' out of the adjoint."""
    n = prev_attrs.shape[1]
    dev = prev_attrs.device
    rast = Rasterizer(n, [cams[0]], tile=cfg.tile, sh_degree=cfg.sh_degree, dilation=cfg.dilation, bg=cfg.bg,
                      device=dev, capacity=capacity)
    d = torch.zeros(2, n, device=dev)
    scratch = torch.zeros_like(prev_attrs)
    gimg = torch.empty_like(rast.images[0])
    for v, c in enumerate(cams):
        rast.set_cameras([c])
        rast.forward(prev_attrs)
        cnt = gimg.numel()
        qg.qg_scaled_diff(cnt, gt_prev[v], gt_cur[v], 2.0 / cnt, gimg)
        rast.backward(prev_attrs, [gimg], scratch, grad_xy=[d])
    return d


def gate_init(d: torch.Tensor, cfg: FitConfig = FitConfig()):
    """Gate logits from d (Eq. 10), the Eq. 10 probabilities and the median norm."""
    n = d.shape[1]
    a = torch.empty(n, device=d.device)
    p = torch.empty(n, device=d.device)
    med = torch.empty(1, device=d.device)
    wsb = qg.qg_gate_init_workspace_size(n)
    ws = torch.empty(wsb, dtype=torch.uint8, device=d.device)
    qg.qg_gate_init(n, d, cfg.gamma0, cfg.gamma1, cfg.tau, a, p, med, ws, wsb)
    return a, p, med
