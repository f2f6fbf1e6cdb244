"""Closed-form and edge cases of Eq. 2 through the HIP path (qg_render_fwd, qg_render_bwd), against the oracle.

* the 0.99 alpha clamp: a single sigma(10) splat centred on a pixel (alpha = 0.99, T = 0.01), and a whole-chain
  scene in which a tenth of the Gaussians have opacity logits ~ N(6, 1), so the forward clamp and the adjoint's
  zero-gradient branch of the clamped side are both compared with the oracle;
* termination: 14 splats with alpha = 1/2 exactly on one pixel centre give 13 contributors, T = 2^-13 and
  image (1 - 2^-13) c, bit-exact;
* the footprint: an isotropic sigma' = 4 px, opacity 1/2 splat reaches alpha >= 1/255 on exactly 489 pixel
  centres, both from 2D records and from a 3D Gaussian through the projection (with no dilation).
"""
import numpy as np
import pytest
import torch

from _helpers import cams_small, keep_mask, rel_l2, small_scene, to_dev
from oracle import composite as OC
from oracle import render as OR
from paper_2412_04469_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qgm():
    from paper_2412_04469_amd import qg, raster
    qg.lib()
    return qg, raster


def _records(rast, sp, W, H, tile):
    """2D splat records written straight into the projected buffers; rectangles cover the whole image."""
    n = len(sp["opacity"])
    rec = np.zeros((n, 12), np.float32)
    rec[:, 0:2] = sp["xy"]
    rec[:, 2] = sp["opacity"]
    rec[:, 4:7] = sp["conic"]
    rec[:, 8:11] = sp["rgb"]
    gw, gh = -(-W // tile[0]), -(-H // tile[1])
    b = rast.proj[0]
    b["splat"].copy_(to_dev(rec))
    b["rect"].copy_(to_dev(np.tile(np.array([0, 0, gw, gh], np.int32), (n, 1)), torch.int32))
    b["ntiles"].copy_(to_dev(np.full(n, gw * gh, np.int32), torch.int32))
    b["depth"].copy_(to_dev(sp["depth"]))
    b["flags"].zero_()


def _render_records(raster, sp, W, H, tile=(16, 16), bg=(0.0, 0.0, 0.0)):
    cam = synth.make_camera((0, 0, -4), W, H)
    rast = raster.Rasterizer(len(sp["opacity"]), [cam], tile=tile, bg=bg)
    _records(rast, sp, W, H, tile)
    rast.bin()
    if rast.ensure_capacity():
        rast.bin()
    rast.render()
    torch.cuda.synchronize()
    return rast


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_single_clamped_splat(qgm, tile):
    qg, raster = qgm
    W, H = 40, 24
    o = np.float32(1.0 / (1.0 + np.exp(-10.0)))  # sigma(10) = 0.99995
    c = np.array([0.8, 0.3, 0.55], np.float32)
    bg = (0.25, 0.5, 0.75)
    sp = {"xy": np.array([[20.5, 11.5]], np.float32), "conic": np.array([[0.5, 0.0, 0.5]], np.float32),
          "opacity": np.array([o]), "rgb": c[None], "depth": np.array([3.0], np.float32)}
    rast = _render_records(raster, sp, W, H, tile, bg)
    img = rast.images[0].cpu().numpy()
    tf = rast.tfinal[0].cpu().numpy()
    a = np.float32(0.99)
    np.testing.assert_allclose(tf[11, 20], 1.0 - 0.99, rtol=1e-5)
    assert tf[11, 20] == np.float32(1.0) - a  # the clamped alpha, bit for bit
    np.testing.assert_allclose(img[:, 11, 20], c * 0.99 + 0.01 * np.array(bg), atol=1e-6)
    # the oracle agrees, and a neighbouring pixel is below the clamp
    ref = OC.composite_image(sp, W, H, bg)
    np.testing.assert_allclose(img, ref["image"], atol=1e-6)
    assert tf[11, 21] > 0.01 + 1e-3


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_termination_after_13_half_alpha_splats_bit_exact(qgm, tile):
    qg, raster = qgm
    W, H = 37, 29
    K = 14
    c = np.array([0.75, 0.5, 0.25], np.float32)  # dyadic: every partial sum is exact in float32
    sp = {"xy": np.tile(np.array([[17.5, 9.5]], np.float32), (K, 1)),
          "conic": np.tile(np.array([[0.3, 0.05, 0.2]], np.float32), (K, 1)),
          "opacity": np.full(K, 0.5, np.float32), "rgb": np.tile(c, (K, 1)),
          "depth": np.linspace(1.0, 5.0, K).astype(np.float32)[::-1].copy()}  # input order is not depth order
    rast = _render_records(raster, sp, W, H, tile)
    img = rast.images[0].cpu().numpy()
    tf = rast.tfinal[0].cpu().numpy()
    last = rast.last[0].cpu().numpy().astype(np.int64)
    assert tf[9, 17] == np.float32(2.0 ** -13)
    assert np.array_equal(img[:, 9, 17], (c * np.float32(1.0 - 2.0 ** -13)).astype(np.float32))
    gw = -(-W // tile[0])
    t = (9 // tile[1]) * gw + 17 // tile[0]
    start = int(rast.ranges[t, 0].item())
    assert last[9, 17] - start == 13  # the 14th (farthest) splat is not added
    vals = rast.vals.cpu().numpy().astype(np.int64)
    assert vals[last[9, 17] - 1] == 1  # depth order: the 13th nearest is input index 1
    ref = OC.composite_image(sp, W, H, (0.0, 0.0, 0.0))
    assert ref["n_contrib"][9, 17] == 13 and ref["t_final"][9, 17] == 2.0 ** -13


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_footprint_489_pixels_from_records(qgm, tile):
    qg, raster = qgm
    W, H = 65, 63
    sp = {"xy": np.array([[32.5, 31.5]], np.float32), "conic": np.array([[1 / 16, 0.0, 1 / 16]], np.float32),
          "opacity": np.array([0.5], np.float32), "rgb": np.ones((1, 3), np.float32),
          "depth": np.array([2.0], np.float32)}
    rast = _render_records(raster, sp, W, H, tile)
    tf = rast.tfinal[0].cpu().numpy()
    assert int((tf < 1.0).sum()) == 489
    yy, xx = np.nonzero(tf < 1.0)
    assert xx.min() == 20 and xx.max() == 44 and yy.min() == 19 and yy.max() == 43


def test_footprint_489_pixels_through_projection(qgm):
    """A 3D Gaussian on the optical axis whose projection is isotropic with sigma' = 4 px (dilation 0)."""
    qg, raster = qgm
    W, H = 65, 63
    f, z0 = 65.0, 5.0
    cam = synth.Camera(f, f, W / 2.0, H / 2.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), W, H)
    s = 4.0 * z0 / f
    planes = np.zeros((59, 1), np.float32)
    planes[0:3, 0] = (0.0, 0.0, z0)
    planes[3, 0] = 1.0
    planes[7:10, 0] = np.log(s)
    planes[10, 0] = 0.0  # opacity 1/2
    planes[11:14, 0] = 1.0
    rast = raster.Rasterizer(1, [cam], tile=(16, 16), dilation=0.0)
    rast.forward(to_dev(planes))
    torch.cuda.synchronize()
    tf = rast.tfinal[0].cpu().numpy()
    assert int((tf < 1.0).sum()) == 489
    assert rast.proj[0]["rect"].cpu().numpy()[0].tolist() == [1, 1, 3, 3]  # pixel span 20..44 at 16x16
    ref = OR.render(planes.astype(np.float64), cam, dilation=0.0)
    assert int((ref["t_final"] < 1.0).sum()) == 489


def _clamped_pixels(sp, idx, W, H, r=3):
    """Number of (Gaussian, pixel centre) pairs among Gaussians idx, within r pixels of the centre, whose raw alpha
    o exp(-q/2) exceeds 0.99 (the clamped side of Eq. 2's alpha)."""
    cnt = 0
    for i in idx:
        if not sp["valid"][i] or sp["opacity"][i] <= 0.99:
            continue
        x, y = sp["xy"][i]
        A, B, C = sp["conic"][i]
        for py in range(int(np.floor(y)) - r, int(np.floor(y)) + r + 1):
            for px in range(int(np.floor(x)) - r, int(np.floor(x)) + r + 1):
                if 0 <= px < W and 0 <= py < H:
                    dx, dy = px + 0.5 - x, py + 0.5 - y
                    q = A * dx * dx + 2 * B * dx * dy + C * dy * dy
                    cnt += int(sp["opacity"][i] * np.exp(-0.5 * q) > 0.99)
    return cnt


def _clamp_scene(seed, n):
    sc = small_scene(seed=seed, n=n, ls_mu=-2.8)
    rng = synth.rng_for(seed + 1000)
    pick = rng.permutation(n)[: n // 10]
    sc.logits[pick] = rng.normal(6.0, 1.0, len(pick)).astype(np.float32)
    return sc, pick


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_clamp_scene_chain_parity(qgm, tile):
    """Forward and adjoint of the whole chain on a scene where a tenth of the Gaussians clamp at alpha = 0.99."""
    qg, raster = qgm
    sc, pick = _clamp_scene(71, 3000)
    cams = cams_small(128, 96)
    bg = (0.2, 0.1, 0.3)
    rast = raster.Rasterizer(sc.n, cams, tile=tile, bg=bg)
    attrs = to_dev(sc.planes())
    rast.forward(attrs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    g_ref = np.zeros((59, sc.n))
    gis = []
    clamp_hits = 0
    for v, cam in enumerate(cams):
        ref0 = OR.render(sc.planes().astype(np.float64), cam, bg)
        keep = keep_mask(ref0)
        print(f"view {v}: {int((~keep).sum())} of {keep.size} pixels excluded by the decision margins")
        assert keep.mean() > 0.99
        # forward parity
        assert np.abs(rast.images[v].cpu().numpy() - ref0["image"])[:, keep].max() <= 1e-4
        assert np.abs(rast.tfinal[v].cpu().numpy() - ref0["t_final"])[keep].max() <= 1e-4
        clamp_hits += _clamped_pixels(ref0["splats"], pick, cam.width, cam.height)
        G = rng.normal(size=(3, cam.height, cam.width)) / (3 * cam.width * cam.height)
        G[:, ~keep] = 0.0
        G = G.astype(np.float32)
        planes = torch.tensor(sc.planes().astype(np.float64), requires_grad=True)
        OR.render(planes, cam, bg, grad_image=G.astype(np.float64))
        g_ref += planes.grad.numpy()
        gis.append(to_dev(G))
    print(f"(Gaussian, pixel) evaluations on the clamped side: {clamp_hits}")
    assert clamp_hits >= 50, clamp_hits  # the clamp is reached at enough pixel centres
    g_attrs = torch.zeros_like(attrs)
    rast.backward(attrs, gis, g_attrs)
    torch.cuda.synchronize()
    g = g_attrs.cpu().numpy()
    groups = {"mean": (0, 3), "quat": (3, 7), "log_scale": (7, 10), "logit": (10, 11), "sh_dc": (11, 14),
              "sh_rest": (14, 59)}
    for name, (lo, hi) in groups.items():
        e = rel_l2(g[lo:hi], g_ref[lo:hi])
        assert e <= 1e-3, (name, e)
    # the clamped Gaussians' own gradients also agree (their opacity gradient comes only from unclamped pixels)
    e = rel_l2(g[:, pick], g_ref[:, pick])
    assert e <= 1e-3, e
