"""Device buffers and autograd glue around the C ABI (no arithmetic of the method happens here).

``Rasterizer`` owns, for a fixed set of cameras and Gaussian count, every buffer that qg_project,
qg_bin, qg_render_fwd and qg_render_bwd need, and enqueues the calls on the current stream.  The bin
capacity grows on demand: after a step whose pair count exceeded the capacity, the step is re-binned.
``RasterizeFn`` and ``DecodeFn`` wrap the hand-written adjoints as ``torch.autograd.Function``s.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import qg


# qg_bin orders each tile list by depth itself (the per-tile route) when capacity <= PER_TILE_AVG * total_tiles;
# above, it sorts the depths of all (view, Gaussian) items first (the depth passes).
PER_TILE_AVG = 512
# The longest list the per-tile route sorts within one workgroup's LDS.  Longer lists are merged through global
# memory by one workgroup each, which takes longer than the depth passes.
PER_TILE_LIST_MAX = 8192


def _u32(shape, device):
    return torch.empty(shape, dtype=torch.int32, device=device)


class Rasterizer:
    def __init__(self, n, cams, tile=(16, 16), sh_degree=3, dilation=0.3, bg=(0.0, 0.0, 0.0), device="cuda",
                 capacity=None, want_keys=False, batch=0, heaviest_first=False):
        self.n = int(n)
        self.cams = list(cams)
        self.V = len(self.cams)
        self.tile_wh = tuple(tile)
        self.batch = int(batch)
        self.heaviest_first = bool(heaviest_first)
        self.tile = qg.tiling(*tile)
        self.sh_degree = int(sh_degree)
        self.dilation = float(dilation)
        self.bg = tuple(float(b) for b in bg)
        self.device = torch.device(device)
        self.want_keys = want_keys
        self.qcams = qg.camera_array(self.cams)
        d = self.device
        n1 = max(self.n, 1)
        self.proj = [{"splat": torch.zeros(n1, qg.SPLAT_STRIDE, device=d),
                      "depth": torch.zeros(n1, device=d),
                      "rect": torch.zeros(n1, 4, dtype=torch.int32, device=d),
                      "ntiles": torch.zeros(n1, dtype=torch.int32, device=d),
                      "flags": torch.zeros(n1, dtype=torch.uint8, device=d)} for _ in range(self.V)]
        self.images = [torch.zeros(3, c.height, c.width, device=d) for c in self.cams]
        self.tfinal = [torch.zeros(c.height, c.width, device=d) for c in self.cams]
        self.last = [_u32((c.height, c.width), d) for c in self.cams]
        self.total_tiles = qg.qg_total_tiles(self.cams, self.tile)
        self.ranges = _u32((self.total_tiles, 2), d)
        self.schedule = None
        if self.heaviest_first:  # blend tiles in heaviest-first order (qg_schedule_tiles after each binning)
            self.schedule = torch.zeros(qg.qg_schedule_words(self.total_tiles), dtype=torch.int32, device=d)
        self.tile = qg.tiling(*tile, batch=self.batch, schedule=self.schedule)
        self.num_pairs = torch.zeros(1, dtype=torch.int64, device=d)
        self.capacity_listeners = []  # called after the pair capacity changed (workspaces that depend on it)
        if capacity is None:
            capacity = max(1024, 16 * self.n * self.V)
        self._alloc_capacity(int(capacity))
        self._tables()

    def _tables(self):
        """ctypes argument tables built once (the calls then only marshal scalars)."""
        self.t_proj = qg.projected_array(self.proj)
        self.t_img = qg._ptr_array(self.images)
        self.t_tf = qg._ptr_array(self.tfinal)
        self.t_last = qg._ptr_array(self.last)

    def set_cameras(self, cams):
        """Switch to other cameras of the same count and resolutions (buffers are reused)."""
        assert len(cams) == self.V
        for a, b in zip(cams, self.cams):
            assert a.width == b.width and a.height == b.height
        self.cams = list(cams)
        self.qcams = qg.camera_array(self.cams)

    def _alloc_capacity(self, cap):
        self.capacity = int(min(cap, 2 ** 32 - 1))
        d = self.device
        self.vals = _u32((max(self.capacity, 1),), d)
        self.keys = torch.empty(max(self.capacity, 1), dtype=torch.int64, device=d) if self.want_keys else None
        self.bin_ws_bytes = qg.qg_bin_workspace_size(self.n, self.V, self.capacity, self.total_tiles)
        self.bin_ws = torch.empty(self.bin_ws_bytes, dtype=torch.uint8, device=d)
        # the adjoint's workspace; in deterministic mode it also holds one set of partials per pair slot
        self.bwd_ws_bytes = qg.qg_render_bwd_workspace_size(self.n, self.V) + self.det_ws_bytes()
        self.bwd_ws = torch.empty(self.bwd_ws_bytes, dtype=torch.uint8, device=d)
        for f in getattr(self, "capacity_listeners", ()):
            f()

    def det_ws_bytes(self) -> int:
        """Workspace the adjoint calls need on top of their own in deterministic mode (0 when it is off)."""
        return qg.qg_deterministic_workspace_size(self.n, self.V, self.capacity) if qg.qg_get_deterministic() else 0

    # -- individual ABI steps -----------------------------------------------------------------
    def project(self, attrs, stream=None):
        qg.qg_project(self.n, attrs.stride(0), attrs, self.sh_degree, self.qcams, self.tile, self.dilation,
                      self.t_proj, stream)

    def bin(self, stream=None, schedule=True):
        """qg_bin, then (heaviest_first, unless schedule=False) the blend order of the new tile lists."""
        qg.qg_bin(self.n, self.t_proj, self.qcams, self.tile, self.capacity, self.vals, self.keys, self.ranges,
                  self.num_pairs, self.bin_ws, self.bin_ws_bytes, stream)
        if schedule:
            self.schedule_tiles(stream)

    def schedule_tiles(self, stream=None):
        """Heaviest-first blend order of the current tile lists (no-op without heaviest_first)."""
        if self.schedule is not None:
            qg.qg_schedule_tiles(self.qcams, self.tile, self.ranges, self.schedule, stream)

    def render(self, stream=None):
        qg.qg_render_fwd(self.t_proj, self.qcams, self.tile, self.vals, self.ranges, self.bg, self.t_img, self.t_tf,
                         self.t_last, stream)

    def render_l1(self, gts, scales, grad_images, partials, stream=None):
        """render, with the L1 term of each view against gts[v] (gradient scale scales[v]) in the same kernel:
        grad_images[v] as qg_l1_loss writes it, partials [2 * total_tiles] float64 per tile."""
        qg.qg_render_fwd_l1(self.t_proj, self.qcams, self.tile, self.vals, self.ranges, self.bg, self.t_img,
                            self.t_tf, self.t_last, gts, scales, grad_images, partials, stream)

    def pair_count(self) -> int:
        """Pair count of the last qg_bin (host sync).  Raises QGError on a negative count, which qg_bin never
        writes: the count buffer (and the tile lists with it) would then be corrupt."""
        p = int(self.num_pairs.item())
        if p < 0:
            raise qg.QGError(qg.QG_ERR_HIP, f"invalid pair count from qg_bin (num_pairs = {p})")
        return p

    def overflowed(self) -> bool:
        """True if the last qg_bin found more pairs than the capacity (host sync; raises as pair_count)."""
        return self.pair_count() > self.capacity

    def longest_list(self) -> int:
        """Entries in the longest tile list of the last qg_bin (host copy of the ranges; 0 after an overflow)."""
        r = self.ranges.cpu().numpy().astype(np.int64)
        return int((r[:, 1] - r[:, 0]).max()) if r.size else 0

    def fit_capacity(self, pairs: int, margin=1.5, longest: int = 0) -> bool:
        """Size the pair capacity for a measured pair count: pairs * margin (at least 1024) when the current one
        leaves less than 5% headroom or is more than 1.25 times that.  If a tile list is longer than
        PER_TILE_LIST_MAX (``longest``, as longest_list gives it), the capacity is kept above
        PER_TILE_AVG * total_tiles, where qg_bin takes the depth passes.  Returns True if the buffers were
        re-allocated."""
        want = max(1024, int(pairs * margin))
        depth_route = PER_TILE_AVG * self.total_tiles + 1
        long_lists = longest > PER_TILE_LIST_MAX
        if long_lists:
            want = max(want, depth_route)
        if (pairs * 1.05 > self.capacity or self.capacity > 1.25 * want
                or (long_lists and self.capacity < depth_route)):
            self._alloc_capacity(want)
            return True
        return False

    def ensure_capacity(self, margin=1.25) -> bool:
        """Host-synchronising check of the last bin; grows the buffers and returns True if it overflowed."""
        p = self.pair_count()
        if p > self.capacity:
            self._alloc_capacity(int(math.ceil(p * margin)))
            return True
        return False

    def forward(self, attrs, stream=None, check=True):
        """project -> bin -> render; returns the list of per-view images [3,H,W]."""
        self.project(attrs, stream)
        self.bin(stream)
        if check and self.ensure_capacity():
            self.bin(stream)
        self.render(stream)
        return self.images

    def backward(self, attrs, grad_images, grad_attrs, grad_xy_abs=None, grad_xy=None, stream=None):
        """Accumulate dL/dattrs (+=) for dL/dimages."""
        qg.qg_render_bwd(self.n, attrs.stride(0), attrs, self.sh_degree, self.qcams, self.tile, self.dilation,
                         self.t_proj, self.vals, self.ranges, self.bg, self.t_tf, self.t_last,
                         [g.contiguous() for g in grad_images], grad_attrs, grad_xy_abs, grad_xy, self.bwd_ws,
                         self.bwd_ws_bytes, stream)


class RasterizeFn(torch.autograd.Function):
    """images = R(attrs) for all cameras of ``rast`` (Eq. 1-2); backward by the hand-written adjoint."""

    @staticmethod
    def forward(ctx, attrs, rast: Rasterizer):
        attrs = attrs.contiguous()
        imgs = rast.forward(attrs)
        ctx.rast = rast
        ctx.save_for_backward(attrs)
        return tuple(im.clone() for im in imgs)

    @staticmethod
    def backward(ctx, *grads):
        (attrs,) = ctx.saved_tensors
        rast = ctx.rast
        g_attrs = torch.zeros_like(attrs)
        gi = [g if g is not None else torch.zeros_like(im) for g, im in zip(grads, rast.images)]
        rast.backward(attrs, gi, g_attrs)
        return g_attrs, None


class DecodeFn(torch.autograd.Function):
    """(attrs, L_reg) = decode(prev, latents, W1, W2, l_p, a) (Eq. 4-8) with the straight-through estimator."""

    @staticmethod
    def forward(ctx, latents, W1, W2, l_p, a, prev, gamma0, gamma1, tau):
        n = prev.shape[1]
        out = torch.empty_like(prev)
        gate = torch.empty(max(n, 1), device=prev.device)
        nb = qg.qg_decode_lreg_blocks(n)
        part = torch.empty(nb, device=prev.device)
        qg.qg_decode_residuals(n, prev.stride(0), prev, latents, latents.shape[0], W1, W2, W1.shape[0], W2.shape[0],
                               l_p, a, gamma0, gamma1, tau, out, gate, part)
        lreg = torch.empty((), device=prev.device)  # Eq. 8 as a mean over the Gaussians, reduced on the device
        qg.qg_decode_lreg_mean(n, part, nb, lreg)
        ctx.save_for_backward(latents, W1, W2, l_p, a)
        ctx.hp = (gamma0, gamma1, tau, n, prev.stride(0))
        return out, lreg

    @staticmethod
    def backward(ctx, g_out, g_lreg):
        latents, W1, W2, l_p, a = ctx.saved_tensors
        gamma0, gamma1, tau, n, ld = ctx.hp
        g_out = torch.zeros((59, ld), device=a.device) if g_out is None else g_out.contiguous()
        gl = torch.zeros_like(latents)
        gW1 = torch.zeros_like(W1)
        gW2 = torch.zeros_like(W2)
        glp = torch.zeros_like(l_p)
        ga = torch.zeros_like(a)
        wsb = qg.qg_decode_bwd_workspace_size(n, latents.shape[0], W1.shape[0], W2.shape[0])
        ws = torch.empty(wsb, dtype=torch.uint8, device=a.device)
        qg.qg_decode_residuals_bwd(n, ld, latents, latents.shape[0], W1, W2, W1.shape[0], W2.shape[0], l_p, a, gamma0,
                                   gamma1, tau, g_out, 0.0, gl, gW1, gW2, glp, ga, ws, wsb)
        if g_lreg is not None:  # the weight of L_reg stays on the device (no host sync)
            qg.qg_decode_lreg_bwd(n, a, gamma0, gamma1, tau, g_lreg.reshape(1).contiguous(), ga)
        return gl, gW1, gW2, glp, ga, None, None, None, None
