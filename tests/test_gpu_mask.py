"""GPU parity of adaptive masked training (Sec. 3.3, "Adaptive Masked Training"): the static/dynamic split, the
dynamic-only render mask, the box dilation and tile flags, the masked L1, and a masked iteration against the
unmasked one."""
import numpy as np
import pytest
import torch

from _helpers import MARGIN_FWD, cams_small, rel_l2, small_scene, to_dev
from oracle import composite as OC
from oracle import mask as OM
from oracle import render as OR
from paper_2412_04469_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qgm():
    from paper_2412_04469_amd import qg, raster
    return qg, raster


def test_dynamic_flags_exact(qgm):
    qg, _ = qgm
    rng = np.random.default_rng(21)
    n = 10007
    d = rng.normal(0.0, 2e-3, (2, n)).astype(np.float32)
    d[:, :50] = 0.0
    d[0, 50:60], d[1, 50:60] = 3e-3, 4e-3  # norm 5e-3 (to float rounding): on the threshold for V = 5, 2 x 2
    for V, W, H in ((1, 2, 2), (3, 2, 2), (4, 2, 2), (5, 2, 2), (20, 1352, 1014), (3, 160, 120)):
        out = torch.empty(n, dtype=torch.uint8, device="cuda")
        qg.qg_dynamic_flags(n, to_dev(d), (W / 2.0) / V, (H / 2.0) / V, 1e-3, out)
        want = OM.dynamic_flags(d, V, W, H, 1e-3)
        assert np.array_equal(out.cpu().numpy().astype(bool), want), V
        assert 0 < want.sum() < n - 50 or (W, H) != (2, 2)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_dynamic_mask_parity(qgm, tile):
    qg, raster = qgm
    sc = small_scene(seed=31, n=3000)
    cams = cams_small(150, 110)
    dyn = np.random.default_rng(3).random(sc.n) < 0.04
    rast = raster.Rasterizer(sc.n, cams, tile=tile)
    rast.forward(to_dev(sc.planes()))
    masks = [torch.full((c.height, c.width), 7, dtype=torch.uint8, device="cuda") for c in cams]
    qg.qg_dynamic_mask(rast.t_proj, rast.qcams, rast.tile, rast.vals, rast.ranges, to_dev(dyn, torch.uint8), masks)
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        sp = dict(OR.render(sc.planes().astype(np.float64), cam)["splats"])
        sp["valid"] = np.asarray(sp["valid"], bool) & dyn
        r = OC.composite_image(sp, cam.width, cam.height)
        want = OM.dynamic_mask(r["t_final"])
        got = masks[v].cpu().numpy()
        assert set(np.unique(got)) <= {0, 1}
        keep = r["margin"] >= MARGIN_FWD
        print(f"[margins] view {v}: {int(keep.size - keep.sum())} of {keep.size} pixels excluded", flush=True)
        assert keep.mean() > 0.99, keep.mean()
        assert np.array_equal(got.astype(bool)[keep], want[keep])
        assert 0.05 < want.mean() < 0.95, want.mean()


def _two_views():
    return [synth.make_camera((0.0, 0.0, -4.0), 200, 150, f=200), synth.make_camera((1.0, 0.0, -4.0), 120, 90, f=120)]


@pytest.mark.parametrize("k", [48, 5, 1])
@pytest.mark.parametrize("tile", [(16, 16), (32, 8)])
def test_dilate_and_tile_flags_exact(qgm, tile, k):
    qg, _ = qgm
    cams = _two_views()
    rng = np.random.default_rng(k)
    masks, want_d, want_f = [], [], []
    for c in cams:
        m = rng.random((c.height, c.width)) < 0.0015
        m[c.height - 1, c.width - 1] = True  # a corner pixel: clipped window
        masks.append(m)
        dd = OM.dilate(m, k)
        want_d.append(dd)
        want_f.append(OM.tile_flags(dd, tile[0], tile[1]))
    t = qg.tiling(*tile)
    dm = [to_dev(m, torch.uint8) for m in masks]
    tmp = [torch.empty_like(x) for x in dm]
    dil = [torch.full_like(x, 9) for x in dm]
    total = qg.qg_total_tiles(cams, t)
    flags = torch.full((total,), 9, dtype=torch.uint8, device="cuda")
    qg.qg_dilate_mask(cams, t, k, dm, tmp, dil, flags)
    torch.cuda.synchronize()
    for v in range(2):
        assert np.array_equal(dil[v].cpu().numpy().astype(bool), want_d[v])
        assert set(np.unique(dil[v].cpu().numpy())) <= {0, 1}
    assert np.array_equal(flags.cpu().numpy().astype(bool), np.concatenate(want_f))
    assert 0 < np.concatenate(want_f).sum() < total


@pytest.mark.parametrize("H,W", [(97, 131),   # plane not a multiple of 4: per-element path
                                 (64, 100)])  # float4 path on 4 whole blocks, per-element tail
def test_masked_l1_parity(qgm, H, W):
    qg, _ = qgm
    rng = np.random.default_rng(8 + H)
    img = rng.random((3, H, W)).astype(np.float32)
    gt = rng.random((3, H, W)).astype(np.float32)
    gt[:, 10, :20] = img[:, 10, :20]  # zero differences: sign 0
    pm = rng.random((H, W)) < 0.3
    count = 3 * H * W
    grad = torch.full((3, H, W), 5.0, device="cuda")
    parts = torch.empty(2 * qg.qg_loss_blocks(count), dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    qg.qg_l1_loss_masked(count, H * W, to_dev(img), to_dev(gt), to_dev(pm, torch.uint8), 1.0, grad, parts)
    qg.qg_loss_reduce(count, parts, out)
    loss, g = OM.masked_l1(img, gt, pm)
    assert abs(float(out[0].item()) - loss) <= 1e-6 * loss
    gg = grad.cpu().numpy()
    assert np.array_equal(gg == 0.0, g == 0.0)
    np.testing.assert_allclose(gg, g, rtol=1e-7, atol=0)
    # every pixel set: the unmasked loss; on the float4 path its sums, in the same order, bit for bit
    ones = torch.ones((H, W), dtype=torch.uint8, device="cuda")
    out1 = torch.empty(2, dtype=torch.float64, device="cuda")
    qg.qg_l1_loss_masked(count, H * W, to_dev(img), to_dev(gt), ones, 1.0, grad, parts)
    qg.qg_loss_reduce(count, parts, out1)
    g1 = grad.clone()
    out2 = torch.empty(2, dtype=torch.float64, device="cuda")
    qg.qg_l1_loss(count, to_dev(img), to_dev(gt), 1.0, grad, parts)
    qg.qg_loss_reduce(count, parts, out2)
    assert torch.equal(g1, grad)
    if (H * W) % 4 == 0:
        assert torch.equal(out1, out2)
    else:
        assert torch.allclose(out1, out2, rtol=1e-6, atol=0)


def _masked_run(qg, raster, sc, cams, tile, bg, gts, pix, flags):
    """project -> bin -> (empty the ranges of unflagged tiles) -> render -> masked L1 -> blend and
    projection adjoints; returns images, T_final, image gradients and dL/dattrs."""
    rast = raster.Rasterizer(sc.n, cams, tile=tile, bg=bg)
    attrs = to_dev(sc.planes())
    rast.project(attrs)
    rast.bin()
    if flags is not None:
        qg.qg_mask_tile_ranges(rast.total_tiles, rast.ranges, flags)
    rast.render()
    parts = torch.empty(2 * qg.qg_loss_blocks(3 * cams[0].width * cams[0].height), dtype=torch.float64,
                        device="cuda")
    gis = []
    for v, c in enumerate(cams):
        G = torch.empty_like(rast.images[v])
        qg.qg_l1_loss_masked(G.numel(), c.width * c.height, rast.images[v], gts[v], pix[v], 1.0, G, parts)
        gis.append(G)
    g = torch.zeros_like(attrs)
    rast.backward(attrs, gis, g)
    torch.cuda.synchronize()
    return ([x.cpu().numpy() for x in rast.images], [x.cpu().numpy() for x in rast.tfinal],
            [x.cpu().numpy() for x in gis], g.cpu().numpy())


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_masked_iteration_matches_unmasked(qgm, tile):
    """With the image gradient zero outside the dilated mask, skipping the unflagged tiles changes nothing
    on the flagged ones (bitwise) and nothing in dL/dattrs (up to the order of float atomics); the skipped
    tiles show the background.  All flags set: the unmasked iteration."""
    qg, raster = qgm
    sc = small_scene(seed=41, n=2500)
    cams = cams_small(160, 120)
    bg = (0.2, 0.1, 0.3)
    rng = np.random.default_rng(12)
    gts = [to_dev(rng.random((3, c.height, c.width)).astype(np.float32)) for c in cams]
    t = qg.tiling(*tile)
    seeds = [np.zeros((c.height, c.width), bool) for c in cams]
    seeds[0][30, 40] = True
    seeds[1][90, 130] = True
    seeds[1][10, 10] = True
    pix = [torch.empty(c.height, c.width, dtype=torch.uint8, device="cuda") for c in cams]
    tmp = [torch.empty_like(p) for p in pix]
    total = qg.qg_total_tiles(cams, t)
    flags = torch.empty(total, dtype=torch.uint8, device="cuda")
    qg.qg_dilate_mask(cams, t, 48, [to_dev(s, torch.uint8) for s in seeds], tmp, pix, flags)
    fl = flags.cpu().numpy().astype(bool)
    assert 0 < fl.sum() < total
    ref = _masked_run(qg, raster, sc, cams, tile, bg, gts, pix, None)
    got = _masked_run(qg, raster, sc, cams, tile, bg, gts, pix, flags)
    off = 0
    for v, c in enumerate(cams):
        gw, gh = -(-c.width // tile[0]), -(-c.height // tile[1])
        tf = fl[off:off + gw * gh].reshape(gh, gw)
        off += gw * gh
        on = np.kron(tf, np.ones((tile[1], tile[0]), bool))[:c.height, :c.width]
        assert np.array_equal(got[0][v][:, on], ref[0][v][:, on])
        assert np.array_equal(got[1][v][on], ref[1][v][on])
        assert np.all(got[1][v][~on] == 1.0)
        for ch in range(3):
            assert np.all(got[0][v][ch][~on] == np.float32(bg[ch]))
        assert np.array_equal(got[2][v], ref[2][v])
        assert not ref[2][v][:, ~on].any()
    assert rel_l2(got[3], ref[3]) <= 1e-5
    assert np.abs(ref[3]).max() > 0
    # every tile flagged: the plain iteration, bit for bit in the images
    allon = torch.ones(total, dtype=torch.uint8, device="cuda")
    same = _masked_run(qg, raster, sc, cams, tile, bg, gts, pix, allon)
    for v in range(len(cams)):
        assert np.array_equal(same[0][v], ref[0][v])


def test_fitter_masks_and_masked_steps(qgm):
    """GateInitializer.masks on a localised change: the mask covers the changed region but not the whole image,
    and a masked step with every tile and pixel set is the plain step (the loss to its summation order, the
    parameters to the order of float atomics)."""
    qg, _ = qgm
    from paper_2412_04469_amd.fit import FitConfig, FrameFitter, GateInitializer, render_views
    wl = synth.workload_fit_local(n=4000, width=160, height=120, n_views=3, frac_move=0.05)
    cfg = FitConfig()
    prev = to_dev(wl.scene.planes())
    gts_prev = render_views(prev, wl.cams, cfg)
    gts = render_views(to_dev(wl.target_scene.planes()), wl.cams, cfg)
    gi = GateInitializer(wl.scene.n, wl.cams, cfg)
    a = gi(prev, gts_prev, gts)
    masks = gi.masks(prev)
    torch.cuda.synchronize()
    dyn = gi.dyn.cpu().numpy().astype(bool)
    assert dyn.any() and not dyn.all()
    for pix, fl in masks:
        assert 0 < int(fl.sum().item()) < fl.numel()
        assert 0 < int(pix.sum().item()) < pix.numel()
    runs = []
    for masked in (False, True):
        f = FrameFitter(prev, wl.cams, gts, cfg)
        f.size_capacity()
        f.reset_frame(a_init=a)
        f.set_masks([(torch.ones_like(p), torch.ones_like(t)) for p, t in masks])
        f.step(1, masked=masked)
        runs.append((f.loss_value(), f.lat.cpu().numpy().copy(), f.a.cpu().numpy().copy()))
    # same image gradient; the loss partials are summed in another order (float4 groups in the plain L1)
    assert abs(runs[1][0] - runs[0][0]) <= 1e-6 * runs[0][0]
    assert rel_l2(runs[1][1], runs[0][1]) <= 1e-5 and rel_l2(runs[1][2], runs[0][2]) <= 1e-5
