"""Per-frame residual fitting (Sec. 3.2-3.4, Eq. 4-11) driven entirely through the C ABI.

One optimiser iteration on one training view (one epoch covers all views, Sec. 4.1) enqueues:
    qg_decode_project -> qg_bin -> qg_render_fwd_l1 (blend and L1 term) -> qg_render_decode_bwd -> qg_adam_multi
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
    batch: int = 0  # blend LDS batch depth (0 = 64)
    heaviest_first: bool = True  # blend tiles in heaviest-first order (a scheduling choice; results unchanged)
    sh_degree: int = 3
    dilation: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)
    # batched steps (BatchedFitter): at most this many views per optimiser step, and a factor on every learning
    # rate (a step over several views has a lower-variance gradient and can take a longer step)
    group_views: int = 16
    batched_lr_scale: float = 1.0
    # adaptive masked training (Sec. 3.3; appendix): dynamic if the view-mean score ||d|| exceeds t_d; the
    # dynamic-only render's mask is dilated by a mask_dilate x mask_dilate box; the first mask_fraction of a
    # frame's iterations render and backpropagate only the tiles holding masked pixels
    t_d: float = 1e-3
    mask_dilate: int = 48
    mask_fraction: float = 0.0
    # Eq. 3's D-SSIM weight lambda (not given in the paper; 3D-GS uses 0.2); 0 fits the L1 term alone
    lambda_dssim: float = 0.0
    # the stochastic hard concrete gate (Eq. 6 as written is deterministic; this draws the gate's logistic noise
    # per Gaussian and step from a counter-based generator seeded by gate_seed); evaluation stays deterministic
    stochastic_gate: bool = False
    gate_seed: int = 2412
    # per-frame densification (3D-GS's stage run inside each frame's fit; implementation details of the paper:
    # from epoch 6 until 80% of the epochs, every 2 epochs, gradient threshold 0.00125), clone below
    # percent_dense x the camera extent, split above, prune opacity below min_opacity (FrameFitter.densify)
    densify: bool = False
    densify_threshold: float = 0.00125
    densify_start_epoch: int = 6
    densify_stop_frac: float = 0.8
    densify_every: int = 2
    percent_dense: float = 0.01
    min_opacity: float = 0.005
    densify_seed: int = 4469
    # the residual decoder: "mlp" (the shared 8 -> 32 -> 56 SiLU MLP of the workload) or "linear" (Eq. 5 as
    # written: one linear decoder per category with the quantisation table's latent dimensions and learning
    # rates, N3DV column: rotation, scaling, opacity, colour base, colour frequencies)
    decoder: str = "mlp"
    paper_dims: tuple = (6, 8, 3, 8, 4)
    paper_latent_lrs: tuple = (0.025, 0.01, 0.05, 0.0125, 0.000625)
    paper_decoder_lrs: tuple = (1e-3, 1e-4, 1e-4, 1e-3, 1e-3)


PAPER_OUT = (4, 3, 1, 3, 45)  # residual planes per category: rotation, scaling, opacity, colour base, frequencies


def xavier_linear_decoder(seed: int, dims, gain=0.1):
    """Packed per-category decoders D_c [M_c][L_c], uniform within gain x the Xavier bound, from a fixed seed.
    With integer latents a latent unit moves an attribute by a column of D_c; at the full Xavier bound (~1 for the
    opacity block) every latent that first rounds to +-1 jumps its Gaussian far, and the fit diverges, while a
    tenth of it gives steps of a few hundredths."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2412, 4469, 2000 + seed])))
    parts = []
    for L, M in zip(dims, PAPER_OUT):
        a = gain * math.sqrt(6.0 / (L + M))
        parts.append(rng.uniform(-a, a, size=(M, L)).astype(np.float32).ravel())
    return np.concatenate(parts)


def xavier_decoder(seed: int, L=8, H=32, M=56):
    """Xavier-uniform W1 [H][L], W2 [M][H] from a fixed seed (decoders need non-zero weights at frame 1)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2412, 4469, 1000 + seed])))
    a1 = math.sqrt(6.0 / (L + H))
    a2 = math.sqrt(6.0 / (H + M))
    return (rng.uniform(-a1, a1, size=(H, L)).astype(np.float32), rng.uniform(-a2, a2, size=(M, H)).astype(np.float32))


class ResidualState:
    """A_{t-1} and the residual parameters of frame t (Eq. 4-8) with their gradients and Adam state."""

    def __init__(self, prev_attrs: torch.Tensor, cfg: FitConfig = FitConfig(), W1=None, W2=None, seed=0,
                 lr_scale=1.0):
        self.cfg = cfg
        # a copy of its own: reset_frame writes each new frame's A_{t-1} here, which must not reach the caller's
        # tensor (a streaming history would otherwise be overwritten)
        self.prev = prev_attrs.detach().clone(memory_format=torch.contiguous_format)
        self.n = int(self.prev.shape[1])
        self.ld = int(self.prev.stride(0))
        dev = self.prev.device
        self.device = dev
        n, L, H = self.n, cfg.latent_dim, cfg.hidden
        self.linear = cfg.decoder == "linear"
        if self.linear:  # Eq. 5 as written: per-category linear decoders (W1 holds the packed D, W2 is unused)
            L = int(sum(cfg.paper_dims))
            if W1 is None:
                W1 = xavier_linear_decoder(seed, cfg.paper_dims)
            self.W1 = torch.as_tensor(W1, device=dev).contiguous()
            self.W2 = torch.zeros(0, device=dev)
        else:
            if W1 is None:
                W1, W2 = xavier_decoder(seed, L, H, 56)
            self.W1 = torch.as_tensor(W1, device=dev).contiguous()
            self.W2 = torch.as_tensor(W2, device=dev).contiguous()
        self.lat = torch.zeros(L, n, device=dev)
        self.lp = torch.zeros(3, n, device=dev)
        self.a = torch.zeros(n, device=dev)
        self.params = {"lat": self.lat, "lp": self.lp, "a": self.a, "W1": self.W1, "W2": self.W2}
        self.lrs = {k: lr * lr_scale for k, lr in (("lat", cfg.lr_latent), ("lp", cfg.lr_pos), ("a", cfg.lr_gate),
                                                   ("W1", cfg.lr_decoder), ("W2", cfg.lr_decoder))}
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.t = 0
        # device step counter {step, 1 - b1^step, 1 - b2^step} for updates that replay from a graph
        self.step_state = torch.zeros(4, dtype=torch.int32, device=dev)
        self.attrs = torch.empty_like(self.prev)
        self.gate = torch.empty(max(n, 1), device=dev)
        # the stochastic gate's logistic noise of the current step (None: the deterministic gate of Eq. 6)
        self.noise = torch.empty(max(n, 1), device=dev) if cfg.stochastic_gate else None
        self.lreg_part = torch.empty(qg.qg_decode_lreg_blocks(n), device=dev)
        if self.linear:
            # one segment per latent category and per decoder block, each with the table's learning rate
            segs = []
            lo = 0
            for Lc, lr in zip(cfg.paper_dims, cfg.paper_latent_lrs):
                sl = slice(lo * n, (lo + Lc) * n)
                segs.append((self.lat.view(-1)[sl], self.grads["lat"].view(-1)[sl], self.m["lat"].view(-1)[sl],
                             self.v["lat"].view(-1)[sl], lr * lr_scale))
                lo += Lc
            segs += [(self.lp, self.grads["lp"], self.m["lp"], self.v["lp"], self.lrs["lp"]),
                     (self.a, self.grads["a"], self.m["a"], self.v["a"], self.lrs["a"])]
            po = 0
            for Lc, Mc, lr in zip(cfg.paper_dims, PAPER_OUT, cfg.paper_decoder_lrs):
                sl = slice(po, po + Lc * Mc)
                segs.append((self.W1[sl], self.grads["W1"][sl], self.m["W1"][sl], self.v["W1"][sl], lr * lr_scale))
                po += Lc * Mc
            self.adam_segs_list = [qg.adam_segments(*[[sg[k] for sg in chunk] for k in range(5)])
                                   for chunk in (segs[:7], segs[7:])]
        else:
            keys = list(self.params)
            self.adam_segs_list = [qg.adam_segments([self.params[k] for k in keys], [self.grads[k] for k in keys],
                                                    [self.m[k] for k in keys], [self.v[k] for k in keys],
                                                    [self.lrs[k] for k in keys])]
        self.adam_segs = self.adam_segs_list[0]

    def reset_frame(self, prev_attrs=None, gts=None, a_init=None, lat_init=None, lp_init=None):
        """New frame: latents and position residuals restart at zero (or at the given initial values), the
        decoder is warm-started, Adam restarts."""
        if prev_attrs is not None:
            self.prev.copy_(prev_attrs)
        if gts is not None:
            self.gts = gts
        for dst, init in ((self.lat, lat_init), (self.lp, lp_init), (self.a, a_init)):
            if init is None:
                dst.zero_()
            else:
                dst.copy_(init)
        for k in self.params:
            self.m[k].zero_()
            self.v[k].zero_()
            self.grads[k].zero_()
        self.step_state.zero_()
        self.t = 0

    def decode(self, stream=None, gate_noise=None):
        """The decoded attributes of frame t (the deterministic gate unless gate_noise is given)."""
        c = self.cfg
        if self.linear:
            qg.qg_decode_linear(self.n, self.ld, self.prev, self.lat, c.paper_dims, self.W1, self.lp, self.a, c.gamma0,
                                c.gamma1, c.tau, self.attrs, self.gate, None, stream, gate_noise=gate_noise)
            return
        qg.qg_decode_residuals(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                               self.lp, self.a, c.gamma0, c.gamma1, c.tau, self.attrs, self.gate, self.lreg_part,
                               stream, gate_noise=gate_noise)

    def adam(self, stream=None, step_state=None, t=None):
        """One Adam step over every parameter segment (clearing the gradients it read); t: the host step count
        of the update (default self.t), unused with step_state."""
        b1, b2 = self.cfg.betas
        t = self.t if t is None else t
        for segs in self.adam_segs_list:
            qg.qg_adam_multi(segs, b1, b2, self.cfg.eps, t, True, stream, step_state=step_state)

    def _eval_psnr(self, rast, cam, gt, loss_part, loss_out, stream=None):
        """PSNR of the decoded frame rendered at ``cam`` against ``gt`` (host sync)."""
        self.decode(stream)
        rast.set_cameras([cam])
        rast.project(self.attrs, stream)
        rast.bin(stream)
        if rast.ensure_capacity():
            rast.bin(stream)
        rast.render(stream)
        cnt = rast.images[0].numel()
        qg.qg_l1_loss(cnt, rast.images[0], gt, 1.0, None, loss_part, stream)
        qg.qg_loss_reduce(cnt, loss_part, loss_out, stream)
        mse = float(loss_out[1].item())
        return float("inf") if mse <= 0 else -10.0 * math.log10(mse)


class FrameFitter(ResidualState):
    """Single-view steps (the plain form): each optimiser iteration renders one training view.

    graph=True (MLP decoder, no densification): the unmasked L1 step of view v runs eagerly the first time and
    is then captured into a graph of its own, which later steps on v replay on the current stream (one graph
    per view: the camera is a launch argument).  Every step then takes the Adam step count and the stochastic
    gate's step from the device counter, and the ground truth is copied into buffers the fitter owns, so that
    a replay reads the current frame's.  Masked and D-SSIM steps still run eagerly."""

    def __init__(self, prev_attrs: torch.Tensor, cams, gts, cfg: FitConfig = FitConfig(), W1=None, W2=None,
                 capacity=None, seed=0, graph=False):
        super().__init__(prev_attrs, cfg, W1, W2, seed)
        self.cams = list(cams)
        # one set of image buffers serves every view
        assert all((c.width, c.height) == (self.cams[0].width, self.cams[0].height) for c in self.cams)
        self.use_graph = bool(graph) and not cfg.densify and not self.linear
        self.graphs = {}
        self.overflows = 0  # training steps found overflowed at a PSNR check (see psnr)
        self.gts = [g.clone() for g in gts] if self.use_graph else gts
        dev = self.device
        n, L, H = self.n, cfg.latent_dim, cfg.hidden
        self.grad_attrs = torch.zeros_like(self.prev)
        if self.linear:  # the paper-mode decoder runs through the unfused calls
            self.dws_bytes = qg.qg_decode_linear_bwd_workspace_size(n, cfg.paper_dims)
        else:
            self.dws_bytes = qg.qg_decode_bwd_workspace_size(n, L, H, 56)
        self.dws = torch.empty(self.dws_bytes, dtype=torch.uint8, device=dev)
        self.fused = not self.linear
        self.rast = Rasterizer(n, [self.cams[0]], tile=cfg.tile, sh_degree=cfg.sh_degree, dilation=cfg.dilation,
                               bg=cfg.bg, device=dev, capacity=capacity, batch=cfg.batch,
                               heaviest_first=cfg.heaviest_first)
        if cfg.densify:  # the densification statistic and the per-view viewspace gradient it is taken from
            self.d_accum = torch.zeros(max(n, 1), device=dev)
            self.d_count = torch.zeros(max(n, 1), device=dev)
            self.d_gxy = torch.zeros(2, max(n, 1), device=dev)
        self._alloc_fws()
        self.rast.capacity_listeners.append(self._alloc_fws)
        self.qcams = [qg.camera_array([c]) for c in self.cams]
        img = self.rast.images[0]
        self.count = img.numel()
        self.grad_img = torch.empty_like(img)
        # the loss partials: per block of qg_l1_loss, or per tile when the blend forward writes the L1 term
        self.loss_part = torch.empty(2 * max(qg.qg_loss_blocks(self.count), self.rast.total_tiles),
                                     dtype=torch.float64, device=dev)
        self.loss_tiles = 0  # tiles of per-tile partials from the last step (0: qg_l1_loss's blocks)
        self.t_gimg = qg._ptr_array([self.grad_img])
        self.t_one = qg.float_array([1.0])
        self.loss_out = torch.zeros(2, dtype=torch.float64, device=dev)
        if cfg.lambda_dssim > 0.0:
            C, H, W = img.shape
            self.ssim_ws_bytes = qg.qg_ssim_workspace_size(C, H, W)
            self.ssim_ws = torch.empty(self.ssim_ws_bytes, dtype=torch.uint8, device=dev)
            self.dssim_out = torch.zeros(1, dtype=torch.float64, device=dev)

    def _alloc_fws(self):
        """The fused adjoint's workspace (plus the deterministic-mode partials, sized by the pair capacity);
        captured graphs hold the addresses of the buffers that were re-allocated, so they are dropped."""
        self.fws_bytes = qg.qg_render_decode_bwd_workspace_size(self.n, 1) + self.rast.det_ws_bytes()
        self.fws = torch.empty(self.fws_bytes, dtype=torch.uint8, device=self.device)
        self.graphs = {}

    def reset_frame(self, prev_attrs=None, gts=None, a_init=None, lat_init=None, lp_init=None):
        if gts is not None and self.use_graph:
            for dst, src in zip(self.gts, gts):
                dst.copy_(src)
            gts = None
        super().reset_frame(prev_attrs, gts, a_init, lat_init, lp_init)

    # -- the step ------------------------------------------------------------------------------
    def forward_view(self, v, stream=None):
        self.rast.qcams = self.qcams[v]
        self.rast.project(self.attrs, stream)
        self.rast.bin(stream)
        self.rast.render(stream)
        return self.rast.images[0]

    def set_masks(self, masks):
        """Per-view (dilated pixel mask [H][W] u8, tile flags u8) from GateInitializer.masks, for masked steps."""
        self.masks = masks

    def step(self, v, stream=None, masked=False, eager=False):
        """One optimiser iteration on training view v (enqueue only).  masked: render and backpropagate only the
        tiles flagged in view v's mask, with the L1 over its masked pixels (Sec. 3.3).  With graph=True an
        unmasked L1 step replays view v's graph (captured after its first, eager, step) unless eager is set."""
        c = self.cfg
        if self.use_graph and not masked and c.lambda_dssim == 0.0:
            g = None if eager else self.graphs.get(v)
            if g is not None:
                g.replay()
            else:
                self._enqueue(v, stream, False)
                if not eager:
                    self.capture(v)
            self.t += 1
            return
        self._enqueue(v, stream, masked)
        self.t += 1

    def capture(self, v):
        """Capture view v's step into its graph (recorded, not run).  The library's kernels must have been
        launched once before (any eager step does that)."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._enqueue(v, None, False)
        self.graphs[v] = g

    def _enqueue(self, v, stream, masked):
        c = self.cfg
        r = self.rast
        dev_step = self.step_state if self.use_graph else None  # the step count on the device (graph mode)
        if self.noise is not None:
            qg.qg_gate_noise(self.n, c.gate_seed, self.t, self.noise, step_state=dev_step, stream=stream)
        fused_l1 = self.fused and not masked and c.lambda_dssim == 0.0  # blend and L1 term in one kernel
        if self.fused:
            r.qcams = self.qcams[v]
            qg.qg_decode_project(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                                 self.lp, self.a, c.gamma0, c.gamma1, c.tau, c.sh_degree, r.qcams, r.tile, c.dilation,
                                 r.t_proj, self.attrs, self.gate, None, stream, gate_noise=self.noise)
            r.bin(stream, schedule=not masked)
            if masked:  # the blend order is taken over the masked tile lists
                qg.qg_mask_tile_ranges(r.total_tiles, r.ranges, self.masks[v][1], stream)
                r.schedule_tiles(stream)
            if fused_l1:
                r.render_l1(qg._ptr_array([self.gts[v]]), self.t_one, self.t_gimg, self.loss_part, stream)
            else:
                r.render(stream)
        else:
            assert not masked, "masked steps use the fused path"
            self.decode(stream, gate_noise=self.noise)
            self.forward_view(v, stream)
        self.loss_tiles = r.total_tiles if fused_l1 else 0
        if masked:
            assert c.lambda_dssim == 0.0, "masked steps fit the L1 term"
            pix = self.masks[v][0]
            qg.qg_l1_loss_masked(self.count, pix.numel(), r.images[0], self.gts[v], pix, 1.0, self.grad_img,
                                 self.loss_part, stream)
        elif c.lambda_dssim > 0.0:
            # Eq. 3: (1 - lambda) L1 + lambda D-SSIM (the D-SSIM gradient is added to the L1 one)
            qg.qg_l1_loss(self.count, r.images[0], self.gts[v], 1.0 - c.lambda_dssim, self.grad_img,
                          self.loss_part, stream)
            C, H, W = r.images[0].shape
            qg.qg_ssim_loss(C, H, W, r.images[0], self.gts[v], c.lambda_dssim, self.grad_img, self.dssim_out,
                            self.ssim_ws, self.ssim_ws_bytes, stream)
        elif not fused_l1:
            qg.qg_l1_loss(self.count, r.images[0], self.gts[v], 1.0, self.grad_img, self.loss_part, stream)
        # parameter gradients are zero here: they start zeroed and qg_adam_multi clears them after use
        gxy = None
        if c.densify:
            qg.qg_zero(self.d_gxy, self.d_gxy.numel() * 4, stream)
            gxy = [self.d_gxy]
        if self.fused:
            qg.qg_render_decode_bwd(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                                    self.lp, self.a, c.gamma0, c.gamma1, c.tau, c.lambda_reg, c.sh_degree, r.qcams,
                                    r.tile, c.dilation, r.t_proj, r.vals, r.ranges, r.bg, r.t_tf, r.t_last,
                                    [self.grad_img], self.grads["lat"], self.grads["W1"], self.grads["W2"],
                                    self.grads["lp"], self.grads["a"], None, gxy, self.fws, self.fws_bytes, stream,
                                    attrs=self.attrs, gate_noise=self.noise)
        else:
            qg.qg_zero(self.grad_attrs, self.grad_attrs.numel() * 4, stream)
            r.backward(self.attrs, [self.grad_img], self.grad_attrs, grad_xy=gxy, stream=stream)
            if self.linear:
                qg.qg_decode_linear_bwd(self.n, self.ld, self.lat, c.paper_dims, self.W1, self.lp, self.a, c.gamma0,
                                        c.gamma1, c.tau, self.grad_attrs, c.lambda_reg, self.grads["lat"],
                                        self.grads["W1"], self.grads["lp"], self.grads["a"], self.dws, self.dws_bytes,
                                        stream, gate_noise=self.noise)
            else:
                qg.qg_decode_residuals_bwd(self.n, self.ld, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                                           self.lp, self.a, c.gamma0, c.gamma1, c.tau, self.grad_attrs, c.lambda_reg,
                                           self.grads["lat"], self.grads["W1"], self.grads["W2"], self.grads["lp"],
                                           self.grads["a"], self.dws, self.dws_bytes, stream, gate_noise=self.noise)
        if c.densify:
            cam = self.cams[v]
            qg.qg_densify_accumulate(self.n, self.d_gxy, r.proj[0]["ntiles"], cam.width / 2.0, cam.height / 2.0,
                                     self.d_accum, self.d_count, stream)
        self.adam(stream, step_state=dev_step, t=self.t + 1)  # step() counts this update after enqueueing it

    def loss_value(self, stream=None):
        """L1 of the last step (host sync)."""
        if self.loss_tiles:  # per-tile partials of the blend's L1 epilogue
            qg.qg_loss_reduce_parts(self.loss_tiles, self.count, self.loss_part, self.loss_out, stream)
        else:
            qg.qg_loss_reduce(self.count, self.loss_part, self.loss_out, stream)
        return float(self.loss_out[0].item())

    def psnr(self, cam, gt, stream=None):
        """PSNR of the decoded frame rendered at ``cam`` against ``gt`` (host sync).  First checks the last
        training step's binning: if it overflowed, the pair capacity grows for the steps that follow and
        ``overflows`` counts it (that step rendered no entries)."""
        if self.rast.ensure_capacity():
            self.overflows += 1
        self.loss_tiles = 0  # the partials now hold the evaluation view's blocks
        return self._eval_psnr(self.rast, cam, gt, self.loss_part, self.loss_out, stream)

    def size_capacity(self, margin=1.5):
        """Bin every view once (host syncs) and size the pair capacity for all of them."""
        worst = longest = 0
        self.decode()
        for v in range(len(self.cams)):
            self.rast.qcams = self.qcams[v]
            self.rast.project(self.attrs)
            self.rast.bin()
            worst = max(worst, self.rast.pair_count())
            longest = max(longest, self.rast.longest_list())
        self.rast.fit_capacity(worst, margin, longest)
        return worst


def densify_iterations(cfg: FitConfig, iters_per_epoch: int, epochs: int):
    """Iterations (counted before the step runs) at which a frame's fit densifies: the starts of epochs
    densify_start_epoch, + densify_every, ... up to densify_stop_frac of the epochs."""
    last = int(math.floor(cfg.densify_stop_frac * epochs))
    return [e * iters_per_epoch for e in range(cfg.densify_start_epoch, last + 1, cfg.densify_every)]


def camera_extent(cams) -> float:
    """3D-GS's scene extent: 1.1 x the largest distance of a camera centre from their mean."""
    c = np.stack([cam.center() for cam in cams])
    return 1.1 * float(np.linalg.norm(c - c.mean(0), axis=1).max())


def densify_fitter(f: "FrameFitter", extent: float, rnd: int, stream=None):
    """The densification stage inside a frame's fit (3D-GS's clone / split / prune on the viewspace-gradient
    statistic accumulated since the last stage).  Returns (a new FrameFitter over the new Gaussian set, the
    action counts).  Every per-Gaussian array is expanded through the plan on the device: A_{t-1}, the residual
    parameters (copied to every child, so a child decodes like its parent) and their Adam moments (zero for new
    Gaussians); split children then get their offset and scale change; the decoder, its moments and the step
    count carry over.  One host read (the new count), then fresh buffers and capacity for the new size."""
    c = f.cfg
    n, dev = f.n, f.device
    f.decode(stream)  # the current decoded attributes (deterministic gate) decide scales and opacities
    action = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    wsb = qg.qg_densify_plan_workspace_size(n)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    qg.qg_densify_plan(n, f.d_accum, f.d_count, f.attrs, f.ld, c.densify_threshold, c.percent_dense * extent,
                       c.min_opacity, action, offsets, ws, wsb, stream)
    n2 = int(offsets[n].item())
    counts = torch.bincount(action[:n].to(torch.int64), minlength=4).tolist()
    prev2 = torch.empty(59, max(n2, 1), device=dev)
    qg.qg_densify_expand(n, action, offsets, 59, f.prev, f.ld, prev2, prev2.stride(0), 0, stream)
    qg.qg_densify_children(n, action, offsets, f.attrs, f.ld, c.densify_seed, rnd, prev2, prev2.stride(0), stream)
    g = FrameFitter(prev2[:, :n2], f.cams, f.gts, c, W1=f.W1.clone(), W2=f.W2.clone(),
                    capacity=int(f.rast.capacity * max(n2, 1) / max(n, 1)) + 1024)
    for k in ("lat", "lp", "a"):
        src, dst = f.params[k], g.params[k]
        planes = 1 if src.dim() == 1 else src.shape[0]
        lds, ldd = (src.shape[-1], dst.shape[-1])
        qg.qg_densify_expand(n, action, offsets, planes, src, lds, dst, ldd, 0, stream)
        for mom_src, mom_dst in ((f.m[k], g.m[k]), (f.v[k], g.v[k])):
            qg.qg_densify_expand(n, action, offsets, planes, mom_src, lds, mom_dst, ldd, 1, stream)
    for k in ("W1", "W2"):
        g.m[k].copy_(f.m[k])
        g.v[k].copy_(f.v[k])
    g.t = f.t
    g.step_state.copy_(f.step_state)
    if getattr(f, "masks", None) is not None:
        g.set_masks(f.masks)
    g.size_capacity()
    return g, {"keep": counts[0], "clone": counts[1], "split": counts[2], "prune": counts[3], "n_before": n,
               "n_after": n2}


def frame_storage(state: ResidualState, stream=None) -> dict:
    """Bytes that store frame t's residuals after its fit: the quantised latents rANS-coded with one model per
    latent dimension (the models as (symbol, 16-bit frequency) pairs), the position residuals of the Gaussians
    whose gate is non-zero as (uint32 index, 3 float32) records, and the float32 decoder weights."""
    n, L = state.n, state.cfg.latent_dim
    dev = state.lat.device
    sym = torch.empty(n * L, dtype=torch.int8, device=dev)
    hist = torch.empty(L * 256, dtype=torch.int32, device=dev)
    ovf = torch.zeros(1, dtype=torch.int32, device=dev)
    qg.qg_latent_symbols(n, state.lat.stride(0), state.lat, L, sym, hist, ovf, stream)
    nz = int((state.gate != 0).sum().item())
    if int(ovf.item()) != 0:
        raise ValueError("latent symbols outside [-128, 127]")
    sym_h = np.ascontiguousarray(sym.cpu().numpy())
    hist_h = np.ascontiguousarray(hist.cpu().numpy().astype(np.uint32).reshape(L, 256))
    coded = qg.qg_rans_encode(L, sym_h, hist_h)
    model = int(sum(1 + 3 * int((row > 0).sum()) for row in hist_h))
    coo = nz * 16
    dec = 4 * (state.W1.numel() + state.W2.numel())  # the MLP's weights, or the packed per-category decoders
    total = coded.size + model + coo + dec
    return {"latent_bytes": int(coded.size), "model_bytes": model, "position_coo_bytes": coo, "nonzero_gates": nz,
            "decoder_bytes": dec, "total_bytes": int(total), "mb_per_frame": round(total / 1e6, 4),
            "latent_bits_per_symbol": round(8.0 * coded.size / max(n * L, 1), 4)}


def view_groups(V: int, max_views: int = qg.MAX_VIEWS):
    """Consecutive groups of near-equal size, at most max_views each."""
    g = -(-V // max_views)
    base, extra = divmod(V, g)
    out, s = [], 0
    for i in range(g):
        k = base + (1 if i < extra else 0)
        out.append(list(range(s, s + k)))
        s += k
    return out


class BatchedFitter(ResidualState):
    """Multi-view steps: one optimiser iteration covers a group of training views (all views of the timestep
    when there are at most 16; otherwise near-equal consecutive groups taken in turn).  Per step, one
    decode+projection pass writes every view of the group, one binning sorts all of their (tile, depth) keys
    in a shared tile index space (per-view tile offsets), one blend launch and one adjoint launch cover all of
    their tiles, and the loss is the mean over the group's views of the per-view mean L1 (weight 1/V each).
    The step has no host synchronisation and no host-dependent arguments (the Adam step count lives on the
    device), so each group's step is captured once into a graph and replayed.  Blend scheduling (tile shape,
    LDS batch depth, heaviest-first tile order) is chosen per fitter; results do not depend on it."""

    def __init__(self, prev_attrs: torch.Tensor, cams, gts, cfg: FitConfig = FitConfig(), W1=None, W2=None,
                 capacity=None, seed=0, batch=0, heaviest_first=None, graph=True, eval_cam=None):
        super().__init__(prev_attrs, cfg, W1, W2, seed, lr_scale=cfg.batched_lr_scale)
        assert not self.linear, "batched steps use the fused MLP-decoder calls"
        self.cams = list(cams)
        # the captured steps read the ground truth from these buffers: new frames are copied into them
        self.gts = [g.clone() for g in gts]
        self.groups = view_groups(len(self.cams), min(int(cfg.group_views), qg.MAX_VIEWS))
        hf = cfg.heaviest_first if heaviest_first is None else bool(heaviest_first)
        self.batch, self.heaviest_first, self.use_graph = int(batch), hf, bool(graph)
        dev = self.device
        n = self.n
        self.rasts = []
        self.gimgs, self.loss_parts, self.counts, self.view_tiles = [], [], [], []
        for g in self.groups:
            r = Rasterizer(n, [self.cams[v] for v in g], tile=cfg.tile, sh_degree=cfg.sh_degree,
                           dilation=cfg.dilation, bg=cfg.bg, device=dev, capacity=capacity, batch=batch,
                           heaviest_first=hf)
            self.rasts.append(r)
            self.gimgs.append([torch.empty_like(im) for im in r.images])
            self.counts.append([im.numel() for im in r.images])
            # the blend's L1 epilogue writes two partial sums per tile; a view's are its tiles' (consecutive ids)
            self.loss_parts.append(torch.empty(2 * r.total_tiles, dtype=torch.float64, device=dev))
            self.view_tiles.append([qg.qg_total_tiles([self.cams[v]], r.tile) for v in g])
        self.t_gimg = [qg._ptr_array(gl) for gl in self.gimgs]
        self.t_gt = [qg._ptr_array([self.gts[v] for v in g]) for g in self.groups]
        self.t_scale = [qg.float_array([1.0 / len(g)] * len(g)) for g in self.groups]
        self._alloc_fws()
        for r in self.rasts:
            r.capacity_listeners.append(self._alloc_fws)
        self.graphs = [None] * len(self.groups)
        self.next_group = 0
        ec = eval_cam if eval_cam is not None else self.cams[0]
        self.eval_rast = Rasterizer(n, [ec], tile=cfg.tile, sh_degree=cfg.sh_degree, dilation=cfg.dilation,
                                    bg=cfg.bg, device=dev)
        self.eval_part = torch.empty(2 * qg.qg_loss_blocks(self.eval_rast.images[0].numel()), dtype=torch.float64,
                                     device=dev)
        self.eval_out = torch.zeros(2, dtype=torch.float64, device=dev)

    def _alloc_fws(self):
        """One fused-adjoint workspace for every group (deterministic-mode partials sized by the largest pair
        capacity); captured graphs hold its address, so they are dropped."""
        vmax = max(len(g) for g in self.groups)
        self.fws_bytes = (qg.qg_render_decode_bwd_workspace_size(self.n, vmax) +
                          max(r.det_ws_bytes() for r in self.rasts))
        self.fws = torch.empty(self.fws_bytes, dtype=torch.uint8, device=self.device)
        self.graphs = [None] * len(self.groups)

    def reset_frame(self, prev_attrs=None, gts=None, a_init=None, lat_init=None, lp_init=None):
        if gts is not None:
            for dst, src in zip(self.gts, gts):
                dst.copy_(src)
        super().reset_frame(prev_attrs, None, a_init, lat_init, lp_init)

    def _enqueue(self, gi, stream=None):
        c = self.cfg
        r = self.rasts[gi]
        views = self.groups[gi]
        if self.noise is not None:  # drawn from the device step counter, so each replay draws afresh
            qg.qg_gate_noise(self.n, c.gate_seed, 0, self.noise, step_state=self.step_state, stream=stream)
        qg.qg_decode_project(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                             self.lp, self.a, c.gamma0, c.gamma1, c.tau, c.sh_degree, r.qcams, r.tile, c.dilation,
                             r.t_proj, self.attrs, self.gate, None, stream, gate_noise=self.noise)
        r.bin(stream)
        # blend and the L1 term of each view (weight 1/V) in one kernel
        r.render_l1(self.t_gt[gi], self.t_scale[gi], self.t_gimg[gi], self.loss_parts[gi], stream)
        qg.qg_render_decode_bwd(self.n, self.ld, self.prev, self.lat, c.latent_dim, self.W1, self.W2, c.hidden, 56,
                                self.lp, self.a, c.gamma0, c.gamma1, c.tau, c.lambda_reg, c.sh_degree, r.qcams,
                                r.tile, c.dilation, r.t_proj, r.vals, r.ranges, r.bg, r.t_tf, r.t_last,
                                self.t_gimg[gi], self.grads["lat"], self.grads["W1"], self.grads["W2"],
                                self.grads["lp"], self.grads["a"], None, None, self.fws, self.fws_bytes, stream,
                                attrs=self.attrs, gate_noise=self.noise)
        b1, b2 = c.betas
        qg.qg_adam_multi(self.adam_segs, b1, b2, c.eps, 0, True, stream, step_state=self.step_state)

    def _capture(self, gi):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._enqueue(gi)
        self.graphs[gi] = g

    def step(self, stream=None):
        """One optimiser iteration on the next view group (the first call of each group runs eagerly and then
        captures its graph; later calls replay it)."""
        gi = self.next_group
        self.next_group = (gi + 1) % len(self.groups)
        if self.use_graph and self.graphs[gi] is not None:
            self.graphs[gi].replay()
        else:
            self._enqueue(gi, stream)
            if self.use_graph:
                torch.cuda.synchronize()
                self._capture(gi)
        self.t += 1

    def invalidate(self):
        """Drop the captured graphs (after buffers were re-allocated)."""
        self.graphs = [None] * len(self.groups)

    def overflowed(self):
        """True if the last binning of some group exceeded its pair capacity (host sync)."""
        return any([r.overflowed() for r in self.rasts])

    def size_capacity(self, margin=1.5):
        """Bin every group once (host syncs) and size each group's pair capacity; drops captured graphs."""
        self.decode()
        worst = []
        for r in self.rasts:
            r.project(self.attrs)
            r.bin()
            p = r.pair_count()
            worst.append(p)
            r.fit_capacity(p, margin, r.longest_list())
        self.invalidate()
        return worst

    def losses(self, gi=None):
        """Per-view mean L1 of the last step of group gi (host sync)."""
        gi = (self.next_group - 1) % len(self.groups) if gi is None else gi
        out = []
        first = 0
        for cnt, nt in zip(self.counts[gi], self.view_tiles[gi]):
            qg.qg_loss_reduce_parts(nt, cnt, self.loss_parts[gi][2 * first:], self.eval_out)
            out.append(float(self.eval_out[0].item()))
            first += nt
        return out

    def psnr(self, cam, gt, stream=None):
        return self._eval_psnr(self.eval_rast, cam, gt, self.eval_part, self.eval_out, stream)


class AttributeFitter:
    """Direct fit of the attribute planes (no residual decoder): the plain differentiable-rasterizer step that the
    small, batched and dense-overlap workloads time.  One optimiser iteration covers all cameras of the fitter in
    one multi-view launch of each call: qg_project -> qg_bin -> qg_render_fwd_l1 (blend and the per-view L1 term,
    weight 1/V) -> qg_render_bwd -> qg_adam_multi over five parameter groups (means, quaternions, log-scales, opacity logits,
    SH) with the 3D-GS learning rates.  The step has no host synchronisation, so it is captured once as a graph
    and replayed; the pair capacity is sized beforehand (size_capacity)."""

    LRS = (1.6e-4, 1e-3, 5e-3, 5e-2, 2.5e-3)  # means, rotation, scale, opacity, SH
    PLANES = ((0, 3), (3, 7), (7, 10), (10, 11), (11, 59))

    def __init__(self, attrs: torch.Tensor, cams, gts, cfg: FitConfig = FitConfig(), capacity=None, graph=True):
        self.cfg = cfg
        self.attrs = attrs.detach().clone(memory_format=torch.contiguous_format)
        self.n = int(self.attrs.shape[1])
        dev = self.attrs.device
        self.device = dev
        self.cams = list(cams)
        self.gts = [g.clone() for g in gts]
        self.rast = Rasterizer(self.n, self.cams, tile=cfg.tile, sh_degree=cfg.sh_degree, dilation=cfg.dilation,
                               bg=cfg.bg, device=dev, capacity=capacity, batch=cfg.batch,
                               heaviest_first=cfg.heaviest_first)
        self.grad = torch.zeros_like(self.attrs)
        self.m = torch.zeros_like(self.attrs)
        self.v = torch.zeros_like(self.attrs)
        self.step_state = torch.zeros(4, dtype=torch.int32, device=dev)
        ld = self.attrs.stride(0)
        segs = []
        for (lo, hi), lr in zip(self.PLANES, self.LRS):
            sl = slice(lo * ld, hi * ld)
            segs.append((self.attrs.view(-1)[sl], self.grad.view(-1)[sl], self.m.view(-1)[sl], self.v.view(-1)[sl],
                         lr))
        self.adam_segs = qg.adam_segments(*[[sg[k] for sg in segs] for k in range(5)])
        self.gimgs = [torch.empty_like(im) for im in self.rast.images]
        self.counts = [im.numel() for im in self.rast.images]
        # two partial sums per tile from the blend's L1 epilogue; a view's are its tiles' (consecutive ids)
        self.loss_part = torch.empty(2 * self.rast.total_tiles, dtype=torch.float64, device=dev)
        self.view_tiles = [qg.qg_total_tiles([c], self.rast.tile) for c in self.cams]
        self.t_gt = qg._ptr_array(self.gts)
        self.t_gimg = qg._ptr_array(self.gimgs)
        self.t_scale = qg.float_array([1.0 / len(self.cams)] * len(self.cams))
        self.use_graph = bool(graph)
        self.graph = None

    def size_capacity(self, margin=1.5):
        """Bin once (host sync) and size the pair capacity; drops a captured graph."""
        r = self.rast
        r.project(self.attrs)
        r.bin()
        p = r.pair_count()
        r.fit_capacity(p, margin, r.longest_list())
        self.graph = None
        return p

    def _enqueue(self, stream=None):
        r = self.rast
        r.project(self.attrs, stream)
        r.bin(stream)
        r.render_l1(self.t_gt, self.t_scale, self.t_gimg, self.loss_part, stream)
        r.backward(self.attrs, self.gimgs, self.grad, stream=stream)
        b1, b2 = self.cfg.betas
        qg.qg_adam_multi(self.adam_segs, b1, b2, self.cfg.eps, 0, True, stream, step_state=self.step_state)

    def step(self, stream=None):
        if self.use_graph and self.graph is not None:
            self.graph.replay()
            return
        self._enqueue(stream)
        if self.use_graph:
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self._enqueue()
            self.graph = g

    def overflowed(self):
        return self.rast.overflowed()

    def loss(self):
        """Mean over views of the per-view mean L1 of the last step (host sync)."""
        out = torch.zeros(2, dtype=torch.float64, device=self.device)
        tot = 0.0
        first = 0
        for c, nt in zip(self.counts, self.view_tiles):
            qg.qg_loss_reduce_parts(nt, c, self.loss_part[2 * first:], out)
            tot += float(out[0].item())
            first += nt
        return tot / len(self.counts)


def render_views(attrs: torch.Tensor, cams, cfg: FitConfig = FitConfig(), capacity=None):
    """Forward renders of ``attrs`` at each camera (used to make ground-truth frames of synthetic scenes)."""
    out = []
    rasts = {}  # one rasterizer per resolution: its image buffers are sized for it
    for c in cams:
        key = (c.width, c.height)
        if key not in rasts:
            rasts[key] = Rasterizer(attrs.shape[1], [c], tile=cfg.tile, sh_degree=cfg.sh_degree,
                                    dilation=cfg.dilation, bg=cfg.bg, device=attrs.device, capacity=capacity)
        rast = rasts[key]
        rast.set_cameras([c])
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


class GateInitializer:
    """Eq. 9-10 once per frame with buffers kept across frames: per view, render A_{t-1} and run one adjoint
    pass with image gradient 2 (I_{t-1} - I_t) / (3HW) to accumulate d, then the gate logits from d."""

    def __init__(self, n, cams, cfg: FitConfig = FitConfig(), device="cuda", capacity=None):
        self.cfg = cfg
        self.cams = list(cams)
        assert all((c.width, c.height) == (self.cams[0].width, self.cams[0].height) for c in self.cams)
        self.rast = Rasterizer(n, [self.cams[0]], tile=cfg.tile, sh_degree=cfg.sh_degree, dilation=cfg.dilation,
                               bg=cfg.bg, device=device, capacity=capacity)
        self.d = torch.zeros(2, n, device=device)
        self.scratch = torch.zeros(59, n, device=device)
        self.gimg = torch.empty_like(self.rast.images[0])
        self.a = torch.empty(n, device=device)
        self.p = torch.empty(n, device=device)
        self.med = torch.empty(1, device=device)
        self.ws_bytes = qg.qg_gate_init_workspace_size(n)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def __call__(self, prev_attrs, gt_prev, gt_cur):
        c = self.cfg
        n = prev_attrs.shape[1]
        qg.qg_zero(self.d, self.d.numel() * 4)
        cnt = self.gimg.numel()
        for v, cam in enumerate(self.cams):
            self.rast.set_cameras([cam])
            self.rast.forward(prev_attrs)
            qg.qg_scaled_diff(cnt, gt_prev[v], gt_cur[v], 2.0 / cnt, self.gimg)
            self.rast.backward(prev_attrs, [self.gimg], self.scratch, grad_xy=[self.d])
        qg.qg_gate_init(n, self.d, c.gamma0, c.gamma1, c.tau, self.a, self.p, self.med, self.ws, self.ws_bytes)
        return self.a

    def masks(self, prev_attrs):
        """Adaptive masked training (Sec. 3.3), after __call__ has accumulated d: the dynamic Gaussians
        (||d|| / V > t_d, d in normalised device coordinates: pixels times (W/2, H/2)), then per view the pixels their render alone reaches (tile lists of A_{t-1}), dilated
        by the mask_dilate box, and the flags of the tiles holding them.  Returns [(pixel mask, tile flags)]."""
        c = self.cfg
        n = prev_attrs.shape[1]
        dev = prev_attrs.device
        if not hasattr(self, "dyn"):
            self.dyn = torch.empty(n, dtype=torch.uint8, device=dev)
            cam0 = self.cams[0]
            self.raw = torch.empty(cam0.height, cam0.width, dtype=torch.uint8, device=dev)
            self.tmp = torch.empty_like(self.raw)
            self.mask_bufs = [(torch.empty_like(self.raw), torch.empty(self.rast.total_tiles, dtype=torch.uint8,
                                                                       device=dev)) for _ in self.cams]
        cam0, V = self.cams[0], len(self.cams)
        qg.qg_dynamic_flags(n, self.d, (cam0.width / 2.0) / V, (cam0.height / 2.0) / V, c.t_d, self.dyn)
        r = self.rast
        for v, cam in enumerate(self.cams):
            r.set_cameras([cam])
            r.project(prev_attrs)
            r.bin()
            if r.ensure_capacity():
                r.bin()
            qg.qg_dynamic_mask(r.t_proj, r.qcams, r.tile, r.vals, r.ranges, self.dyn, [self.raw])
            pix, flags = self.mask_bufs[v]
            qg.qg_dilate_mask(r.qcams, r.tile, c.mask_dilate, [self.raw], [self.tmp], [pix], flags)
        return self.mask_bufs


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
