"""Parity of the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerances: images and T_final within 1e-4 absolute, gradients within 1e-3 relative L2 per attribute
group, integer outputs (tile rectangles, sorted keys/values, ranges, pair counts, last contributor)
bit-exact.  Pixels whose oracle decision margin (1/255 skip, 0.99 clamp, T < 1e-4 stop, order of two
adjacent depths) is below MARGIN_FWD may decide differently in float32 and are excluded and counted.
"""
import numpy as np
import pytest
import torch

from _helpers import MARGIN_FWD, cams_small, keep_mask, rel_l2, small_scene, splat_fields, to_dev
from oracle import binning as OB
from oracle import composite as OC
from oracle import decode as OD
from oracle import loss as OL
from oracle import project as OP
from oracle import render as OR
from paper_2412_04469_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qgm():
    from paper_2412_04469_amd import qg, raster
    qg.lib()
    return qg, raster


def _oracle_proj(scene, cam, deg=3, dil=0.3):
    return OP.project(*OP.scene_tensors(scene), cam, deg, dil)


@pytest.mark.parametrize("deg", [3, 2, 1, 0])
def test_project_parity(qgm, deg):
    qg, raster = qgm
    sc = small_scene(seed=11, n=3000)
    cams = cams_small()
    rast = raster.Rasterizer(sc.n, cams, tile=(16, 16), sh_degree=deg)
    attrs = to_dev(sc.planes())
    rast.project(attrs)
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        g = splat_fields(rast.proj[v])
        o = _oracle_proj(sc, cam, deg)
        valid = o["valid"].numpy()
        gvalid = (g["flags"] & 0x80) == 0
        assert np.array_equal(valid, gvalid)
        assert valid.sum() > 1000
        np.testing.assert_allclose(g["xy"][valid], o["xy"].detach().numpy()[valid], rtol=1e-5, atol=2e-4)
        np.testing.assert_allclose(g["depth"][valid], o["depth"].detach().numpy()[valid], rtol=1e-6)
        np.testing.assert_allclose(g["opacity"][valid], o["opacity"].detach().numpy()[valid], rtol=1e-6)
        np.testing.assert_allclose(g["rgb"][valid], o["rgb"].detach().numpy()[valid], rtol=1e-5, atol=1e-5)
        # the conic to 1e-5 relative to its largest entry (the 2D part runs in double precision, stored as float32)
        oc = o["conic"].detach().numpy()[valid]
        scale = np.abs(oc).max(1, keepdims=True)
        np.testing.assert_allclose(g["conic"][valid] / scale, oc / scale, atol=1e-5)
        rect, nt, edges = OP.tile_rect(o["xy"].detach().numpy(), o["cov2d"].detach().numpy(),
                                       o["opacity"].detach().numpy(), valid, cam.width, cam.height, 16, 16)
        near = (np.abs(edges - np.round(edges)) < 1e-4).any(1) & valid
        ok = ~near
        assert np.array_equal(g["rect"][ok], rect[ok])
        assert np.array_equal(g["ntiles"][ok], nt[ok])
        assert near.sum() <= 0.01 * valid.sum()
        # colour-clamp bits agree where the pre-clamp value is not at rounding distance of 0
        pre = o["rgb_pre"].detach().numpy()
        far = (np.abs(pre) > 1e-5).all(1) & valid
        bits = np.stack([(g["flags"] >> c) & 1 for c in range(3)], 1).astype(bool)
        assert np.array_equal(bits[far], (pre < 0)[far])


def _fill_proj_for_bin(qg, bufs, rect, depth):
    n = len(depth)
    nt = (rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1])
    bufs["rect"].copy_(to_dev(rect, torch.int32))
    bufs["ntiles"].copy_(to_dev(nt.astype(np.int32), torch.int32))
    bufs["depth"].copy_(to_dev(depth))
    bufs["flags"].zero_()
    return nt


def _random_rects(rng, n, gw, gh, empty_frac=0.2, max_w=6):
    x0 = rng.integers(0, gw, n)
    y0 = rng.integers(0, gh, n)
    x1 = np.minimum(x0 + 1 + rng.integers(0, max_w, n), gw)
    y1 = np.minimum(y0 + 1 + rng.integers(0, max_w, n), gh)
    r = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    r[rng.uniform(size=n) < empty_frac] = 0
    return r


@pytest.mark.parametrize("tile,sizes,n", [((16, 16), [(100, 70)], 5000),
                                          ((8, 8), [(100, 70), (64, 64), (33, 17)], 3000),
                                          ((32, 8), [(300, 200), (50, 40)], 20000),
                                          ((16, 16), [(1352, 1014)], 70000),
                                          # > 4M pairs (16 items per thread) and > 65,536 tiles (3 tile passes)
                                          ((8, 8), [(1920, 1080), (1920, 1080), (1352, 1014)], 300000)])
def test_bin_bit_exact(qgm, tile, sizes, n):
    qg, raster = qgm
    rng = synth.rng_for(20 + n)
    cams = [synth.make_camera((0, 0, -4), w, h) for (w, h) in sizes]
    rast = raster.Rasterizer(n, cams, tile=tile, want_keys=True, capacity=64)
    keys_all, vals_all = [], []
    off = 0
    for v, c in enumerate(cams):
        gw, gh = -(-c.width // tile[0]), -(-c.height // tile[1])
        rect = _random_rects(rng, n, gw, gh)
        depth = rng.uniform(0.3, 30.0, n).astype(np.float32)
        depth[rng.integers(0, n, n // 10)] = depth[0]  # equal depths: ties by index
        _fill_proj_for_bin(qg, rast.proj[v], rect, depth)
        k, vv = OB.make_pairs_fast(rect, depth, gw, off)
        keys_all.append(k)
        vals_all.append(vv)
        off += gw * gh
    keys = np.concatenate(keys_all)
    vals = np.concatenate(vals_all)
    ks, vs = OB.sort_pairs(keys, vals)
    ranges = OB.tile_ranges(ks, off)
    # first with a capacity that is too small: overflow reported, nothing emitted, ranges empty
    rast.bin()
    torch.cuda.synchronize()
    assert int(rast.num_pairs.item()) == len(ks)
    assert (rast.ranges.cpu().numpy() == 0).all()
    assert rast.ensure_capacity()
    rast.bin()
    torch.cuda.synchronize()
    for rep in range(3):
        if rep == 1:  # a second call on the same workspace must not see the first one's sort state
            rast.vals.zero_()
            rast.bin()
            torch.cuda.synchronize()
        if rep == 2:
            # a capacity far above the pair count: the radix passes' grids are sized by the capacity (here
            # above 2000 blocks of 4096 pairs) and read the pair count on the device
            rast._alloc_capacity(9 * 2**20 + len(ks))
            rast.bin()
            torch.cuda.synchronize()
        P = int(rast.num_pairs.item())
        assert P == len(ks)
        assert np.array_equal(rast.vals[:P].cpu().numpy().astype(np.uint32), vs)
        assert np.array_equal(rast.keys[:P].cpu().numpy().view(np.uint64), ks)
        assert np.array_equal(rast.ranges.cpu().numpy().astype(np.uint32), ranges)


@pytest.mark.parametrize("layout", ["hot_lds", "hot_global", "many_long", "two_views"])
def test_bin_long_tile_lists(qgm, layout):
    """Short average lists (the per-tile depth order) with tiles far longer than one wavefront sorts:
    hot_lds: 3,000 rectangles share the four centre tiles of a 512x512 view (lists sorted in LDS);
    hot_global: 20,000 do (lists longer than LDS holds, merged through global memory);
    many_long: 1,100 rectangles cover the top 10 tile rows (320 long lists, more than the blocks that sort them);
    two_views: a hot spot in each of two views of different sizes (each long list takes its own view's depths).
    The lists equal the oracle's, and those of the depth-pass path (a capacity far above the average)."""
    qg, raster = qgm
    rng = synth.rng_for(29)
    tile = (16, 16)
    sizes = [(512, 512), (384, 256)] if layout == "two_views" else [(512, 512)]
    cams = [synth.make_camera((0, 0, -4), w, h) for (w, h) in sizes]
    n = {"hot_lds": 20000, "hot_global": 30000, "many_long": 8000, "two_views": 12000}[layout]
    rast = raster.Rasterizer(n, cams, tile=tile, want_keys=True, capacity=64)
    keys_all, vals_all = [], []
    off = 0
    for v, c in enumerate(cams):
        gw, gh = -(-c.width // tile[0]), -(-c.height // tile[1])
        if layout == "many_long":
            rect = _random_rects(rng, n, gw, gh, max_w=2)
            rect[rng.permutation(n)[:1100]] = np.array([0, 0, gw, 10], np.int32)
        else:
            hot_n = {"hot_lds": 3000, "hot_global": 20000, "two_views": 3000 - 500 * v}[layout]
            rect = _random_rects(rng, n, gw, gh, max_w=4)
            cx, cy = gw // 2 - 1, gh // 2 - 1
            rect[rng.permutation(n)[:hot_n]] = np.array([cx, cy, cx + 2, cy + 2], np.int32)
        depth = rng.uniform(0.3, 30.0, n).astype(np.float32)
        depth[rng.integers(0, n, n // 10)] = depth[0]
        _fill_proj_for_bin(qg, rast.proj[v], rect, depth)
        k, vv = OB.make_pairs_fast(rect, depth, gw, off)
        keys_all.append(k)
        vals_all.append(vv)
        off += gw * gh
    ks, vs = OB.sort_pairs(np.concatenate(keys_all), np.concatenate(vals_all))
    ranges = OB.tile_ranges(ks, off)
    lens = np.diff(ranges, axis=1)[:, 0]
    if layout in ("hot_lds", "two_views"):
        assert 2048 < lens.max() <= 8192
    elif layout == "hot_global":
        assert lens.max() > 16384  # three runs of the LDS capacity (8,192)
    else:
        assert (lens > 1024).sum() > 256
    if layout == "two_views":  # a long list in each view
        t0 = -(-sizes[0][0] // tile[0]) * -(-sizes[0][1] // tile[1])
        assert lens[:t0].max() > 1024 and lens[t0:].max() > 1024
    rast.bin()
    assert rast.ensure_capacity()
    assert rast.capacity <= 512 * rast.total_tiles  # the per-tile path
    for cap in (None, 600 * rast.total_tiles):  # then the depth passes
        if cap:
            rast._alloc_capacity(cap)
        rast.bin()
        torch.cuda.synchronize()
        P = int(rast.num_pairs.item())
        assert P == len(ks)
        assert np.array_equal(rast.vals[:P].cpu().numpy().astype(np.uint32), vs), cap
        assert np.array_equal(rast.keys[:P].cpu().numpy().view(np.uint64), ks)
        assert np.array_equal(rast.ranges.cpu().numpy().astype(np.uint32), ranges)


def test_bin_empty(qgm):
    qg, raster = qgm
    cams = [synth.make_camera((0, 0, -4), 64, 48)]
    rast = raster.Rasterizer(0, cams, capacity=16)
    rast.bin()
    torch.cuda.synchronize()
    assert int(rast.num_pairs.item()) == 0
    assert (rast.ranges.cpu().numpy() == 0).all()


def _blend_inputs(qg, rast, sp, cam_w, cam_h, tile):
    """Write 2D splat records straight into the projected buffers, with rectangles covering the whole image."""
    n = len(sp["opacity"])
    rec = np.zeros((n, 12), np.float32)
    rec[:, 0:2] = sp["xy"]
    rec[:, 2] = sp["opacity"]
    rec[:, 4:7] = sp["conic"]
    rec[:, 8:11] = sp["rgb"]
    gw, gh = -(-cam_w // tile[0]), -(-cam_h // tile[1])
    rect = np.tile(np.array([0, 0, gw, gh], np.int32), (n, 1))
    b = rast.proj[0]
    b["splat"].copy_(to_dev(rec))
    _fill_proj_for_bin(qg, b, rect, sp["depth"])


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.25, 0.5, 0.75)])
def test_blend_fwd_parity_and_tiling_invariance(qgm, bg):
    qg, raster = qgm
    W, H, n = 100, 70, 600
    sp = synth.random_splats(synth.rng_for(31), n, W, H, radius_px=(1.0, 10.0), opacity=(0.02, 0.99))
    cam = synth.make_camera((0, 0, -4), W, H)
    ref = OC.composite_image(sp, W, H, bg)
    keep = keep_mask(ref, order=False, margin=1e-5)  # identical float32 records and depths on both sides
    assert keep.mean() > 0.99
    outs = []
    for tile in [(16, 16), (8, 8), (32, 8)]:
        rast = raster.Rasterizer(n, [cam], tile=tile, bg=bg)
        _blend_inputs(qg, rast, sp, W, H, tile)
        rast.bin()
        if rast.ensure_capacity():
            rast.bin()
        rast.render()
        torch.cuda.synchronize()
        img = rast.images[0].cpu().numpy()
        tf = rast.tfinal[0].cpu().numpy()
        last = rast.last[0].cpu().numpy().astype(np.int64)
        vals = rast.vals.cpu().numpy().astype(np.int64)
        gid = np.where(last > 0, vals[np.maximum(last - 1, 0)], -1)
        # a pixel with no contributor has last == its tile start; map those to -1
        starts = rast.ranges.cpu().numpy()[:, 0].astype(np.int64)
        gw = -(-W // tile[0])
        ti = (np.arange(H)[:, None] // tile[1]) * gw + (np.arange(W)[None, :] // tile[0])
        gid = np.where(last == starts[ti], -1, gid)
        assert np.abs(img - ref["image"])[:, keep].max() <= 1e-4
        assert np.abs(tf - ref["t_final"])[keep].max() <= 1e-4
        assert np.array_equal(gid[keep], ref["last_id"][keep])
        outs.append((img, tf))
    for img, tf in outs[1:]:
        assert np.array_equal(img, outs[0][0]) and np.array_equal(tf, outs[0][1])


def _gpu_chain(raster, sc, cams, tile=(16, 16), deg=3, bg=(0.0, 0.0, 0.0)):
    rast = raster.Rasterizer(sc.n, cams, tile=tile, sh_degree=deg, bg=bg)
    attrs = to_dev(sc.planes())
    rast.forward(attrs)
    torch.cuda.synchronize()
    return rast, attrs


def _gid_of_last(rast, v, tile):
    cam = rast.cams[v]
    W, H = cam.width, cam.height
    last = rast.last[v].cpu().numpy().astype(np.int64)
    vals = rast.vals.cpu().numpy().astype(np.int64)
    starts = rast.ranges.cpu().numpy()[:, 0].astype(np.int64)
    gw = -(-W // tile[0])
    gh = -(-H // tile[1])
    off = sum(-(-c.width // tile[0]) * -(-c.height // tile[1]) for c in rast.cams[:v])
    ti = off + (np.arange(H)[:, None] // tile[1]) * gw + (np.arange(W)[None, :] // tile[0])
    gid = np.where(last > 0, vals[np.maximum(last - 1, 0)], -1)
    return np.where(last == starts[ti], -1, gid)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_chain_fwd_parity(qgm, tile):
    qg, raster = qgm
    sc = small_scene(seed=12, n=4000)
    cams = cams_small(150, 110)
    bg = (0.1, 0.2, 0.3)
    rast, _ = _gpu_chain(raster, sc, cams, tile, bg=bg)
    for v, cam in enumerate(cams):
        ref = OR.render(sc.planes().astype(np.float64), cam, bg)
        keep = keep_mask(ref)
        assert keep.mean() > 0.995, keep.mean()
        img = rast.images[v].cpu().numpy()
        assert np.abs(img - ref["image"])[:, keep].max() <= 1e-4
        assert np.abs(rast.tfinal[v].cpu().numpy() - ref["t_final"])[keep].max() <= 1e-4
        gid = _gid_of_last(rast, v, tile)
        assert np.array_equal(gid[keep], ref["last_id"][keep])


def _groups(g):
    return {"mean": g[0:3], "quat": g[3:7], "log_scale": g[7:10], "logit": g[10:11], "sh_dc": g[11:14],
            "sh_rest": g[14:59]}


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_chain_bwd_parity(qgm, tile):
    qg, raster = qgm
    sc = small_scene(seed=13, n=2500)
    cams = cams_small(128, 96)
    bg = (0.2, 0.1, 0.3)
    rast, attrs = _gpu_chain(raster, sc, cams, tile, bg=bg)
    rng = np.random.default_rng(5)
    gis, refs = [], []
    g_ref = np.zeros((59, sc.n))
    gxy_ref = []
    for v, cam in enumerate(cams):
        ref0 = OR.render(sc.planes().astype(np.float64), cam, bg)
        G = rng.normal(size=(3, cam.height, cam.width)) / (3 * cam.width * cam.height)
        G[:, ~keep_mask(ref0)] = 0.0
        G = G.astype(np.float32)
        planes = torch.tensor(sc.planes().astype(np.float64), requires_grad=True)
        ref = OR.render(planes, cam, bg, grad_image=G.astype(np.float64))
        g_ref += planes.grad.numpy()
        gxy_ref.append(ref["g_xy"])
        gis.append(to_dev(G))
    g_attrs = torch.zeros_like(attrs)
    gabs = torch.zeros(sc.n, device="cuda")
    gxy = [torch.zeros(2, sc.n, device="cuda") for _ in cams]
    rast.backward(attrs, gis, g_attrs, gabs, gxy)
    torch.cuda.synchronize()
    g = g_attrs.cpu().numpy()
    for name, gg in _groups(g).items():
        assert rel_l2(gg, _groups(g_ref)[name]) <= 1e-3, (name, rel_l2(gg, _groups(g_ref)[name]))
    for v in range(len(cams)):
        assert rel_l2(gxy[v].cpu().numpy(), gxy_ref[v].T) <= 1e-3
    np.testing.assert_allclose(gabs.cpu().numpy(),
                               sum(np.linalg.norm(x, axis=1) for x in gxy_ref), rtol=1e-3, atol=1e-9)


@pytest.mark.parametrize("n", [5000, 7, 70001])
def test_decode_parity(qgm, n):
    qg, raster = qgm
    rng = synth.rng_for(40)
    prev = rng.normal(size=(59, n)).astype(np.float32)
    lat = rng.normal(0, 1.5, size=(8, n)).astype(np.float32)
    W1 = (rng.normal(size=(32, 8)) * 0.3).astype(np.float32)
    W2 = (rng.normal(size=(56, 32)) * 0.2).astype(np.float32)
    lp = rng.normal(0, 0.1, size=(3, n)).astype(np.float32)
    a = rng.normal(0, 1.0, size=n).astype(np.float32)
    hp = (-0.5, 1.01, 0.3)
    Gout = rng.normal(size=(59, n)).astype(np.float32)
    lam = 0.01
    # oracle (float64, autograd)
    t = lambda x: torch.tensor(x.astype(np.float64), requires_grad=True)
    tl, tW1, tW2, tlp, ta = t(lat), t(W1), t(W2), t(lp), t(a)
    out, g, lreg = OD.decode(torch.tensor(prev.astype(np.float64)), tl, tW1, tW2, tlp, ta, *hp)
    ((out * torch.tensor(Gout.astype(np.float64))).sum() + lam * lreg).backward()
    # GPU
    d = {k: to_dev(x) for k, x in dict(prev=prev, lat=lat, W1=W1, W2=W2, lp=lp, a=a, G=Gout).items()}
    o_g = torch.empty_like(d["prev"])
    gate = torch.empty(n, device="cuda")
    part = torch.empty(qg.qg_decode_lreg_blocks(n), device="cuda")
    qg.qg_decode_residuals(n, n, d["prev"], d["lat"], 8, d["W1"], d["W2"], 32, 56, d["lp"], d["a"], *hp, o_g, gate,
                           part)
    grads = [torch.zeros_like(d[k]) for k in ("lat", "W1", "W2", "lp", "a")]
    wsb = qg.qg_decode_bwd_workspace_size(n, 8, 32, 56)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    qg.qg_decode_residuals_bwd(n, n, d["lat"], 8, d["W1"], d["W2"], 32, 56, d["lp"], d["a"], *hp, d["G"], lam,
                               *grads, ws, wsb)
    torch.cuda.synchronize()
    on = out.detach().numpy()
    scale = np.abs(on - prev) + np.abs(prev) + 1.0
    assert (np.abs(o_g.cpu().numpy() - on) / scale).max() < 2e-6
    np.testing.assert_allclose(gate.cpu().numpy(), g.detach().numpy(), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(part.sum().item() / n, lreg.item(), rtol=1e-5)
    for name, gg, ref in zip(("lat", "W1", "W2", "lp", "a"), grads, (tl, tW1, tW2, tlp, ta)):
        assert rel_l2(gg.cpu().numpy(), ref.grad.numpy()) <= 1e-5, name


@pytest.mark.parametrize("n", [1, 300, 70001])
def test_decode_lreg_mean_and_adjoint_on_device(qgm, n):
    """Eq. 8's mean (qg_decode_lreg_mean) and its gate-logit adjoint with a device weight (qg_decode_lreg_bwd),
    directly and through DecodeFn's autograd, against the oracle's mean and its autograd gradient."""
    qg, raster = qgm
    rng = synth.rng_for(43)
    a = rng.normal(0, 2.0, size=n).astype(np.float32)
    hp = (-0.5, 1.01, 0.3)
    lam = 0.37
    ta = torch.tensor(a.astype(np.float64), requires_grad=True)
    zero = lambda *s: torch.zeros(*s, dtype=torch.float64)
    _, _, lreg = OD.decode(zero(59, n), zero(8, n), zero(32, 8), zero(56, 32), zero(3, n), ta, *hp)
    (lam * lreg).backward()
    d_a = to_dev(a)
    prev = torch.zeros(59, n, device="cuda")
    lat, lp = torch.zeros(8, n, device="cuda"), torch.zeros(3, n, device="cuda")
    W1, W2 = torch.zeros(32, 8, device="cuda"), torch.zeros(56, 32, device="cuda")
    part = torch.empty(qg.qg_decode_lreg_blocks(n), device="cuda")
    qg.qg_decode_residuals(n, n, prev, lat, 8, W1, W2, 32, 56, lp, d_a, *hp, torch.empty_like(prev), None, part)
    mean = torch.empty(1, device="cuda")
    qg.qg_decode_lreg_mean(n, part, part.numel(), mean)
    ga = torch.zeros(n, device="cuda")
    qg.qg_decode_lreg_bwd(n, d_a, *hp, torch.tensor([lam], device="cuda"), ga)
    torch.cuda.synchronize()
    np.testing.assert_allclose(mean.item(), lreg.item(), rtol=1e-6)
    assert rel_l2(ga.cpu().numpy(), ta.grad.numpy()) <= 1e-6
    # the autograd wrapper: same value, same gate gradient, no host read of the weight
    d_a.requires_grad_(True)
    out, lr = raster.DecodeFn.apply(lat, W1, W2, lp, d_a, prev, *hp)
    (lam * lr).backward()
    torch.cuda.synchronize()
    np.testing.assert_allclose(lr.item(), lreg.item(), rtol=1e-6)
    assert rel_l2(d_a.grad.cpu().numpy(), ta.grad.numpy()) <= 1e-6


def test_loss_and_adam_parity(qgm):
    qg, raster = qgm
    rng = synth.rng_for(41)
    img = rng.uniform(-0.2, 1.2, size=(3, 67, 91)).astype(np.float32)
    gt = rng.uniform(0, 1, size=(3, 67, 91)).astype(np.float32)
    gt.ravel()[::97] = img.ravel()[::97]  # exact ties: sign(0) = 0
    cnt = img.size
    d_img, d_gt = to_dev(img), to_dev(gt)
    grad = torch.empty_like(d_img)
    part = torch.empty(2 * qg.qg_loss_blocks(cnt), dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    qg.qg_l1_loss(cnt, d_img, d_gt, 1.0, grad, part)
    qg.qg_loss_reduce(cnt, part, out)
    torch.cuda.synchronize()
    l1, g = OL.l1(img, gt)
    np.testing.assert_allclose(out[0].item(), l1, rtol=1e-6)
    assert np.array_equal(grad.cpu().numpy(), g.astype(np.float32))
    mse = ((np.clip(img.astype(np.float64), 0, 1) - gt) ** 2).mean()
    np.testing.assert_allclose(out[1].item(), mse, rtol=1e-6)
    np.testing.assert_allclose(-10 * np.log10(out[1].item()), OL.psnr(img, gt), rtol=1e-6)
    from oracle import adam as OA
    p = rng.normal(size=1000).astype(np.float32)
    m = np.zeros(1000); v = np.zeros(1000); pp = p.astype(np.float64)
    dp, dm, dv = to_dev(p), torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    for step in range(1, 4):
        gr = rng.normal(size=1000).astype(np.float32)
        qg.qg_adam(1000, dp, to_dev(gr), dm, dv, 0.01, 0.9, 0.999, 1e-8, step)
        pp, m, v = OA.adam_step(pp, gr.astype(np.float64), m, v, step, 0.01)
    torch.cuda.synchronize()
    np.testing.assert_allclose(dp.cpu().numpy(), pp, rtol=1e-5, atol=1e-6)


def test_adam_multi_parity(qgm):
    """Several parameter groups in one launch: each segment follows the oracle's Adam with its own learning rate,
    and its gradient is cleared after the step (uneven sizes, one empty segment)."""
    qg, raster = qgm
    from oracle import adam as OA
    rng = synth.rng_for(43)
    sizes, lrs = [1, 0, 1000, 257, 70001], [0.1, 0.5, 1.6e-4, 0.01, 1e-3]
    ps = [rng.normal(size=n).astype(np.float32) for n in sizes]
    dev_p = [to_dev(p) for p in ps]
    dev_g = [torch.zeros(n, device="cuda") for n in sizes]
    dev_m = [torch.zeros(n, device="cuda") for n in sizes]
    dev_v = [torch.zeros(n, device="cuda") for n in sizes]
    segs = qg.adam_segments(dev_p, dev_g, dev_m, dev_v, lrs)
    ref = [(p.astype(np.float64), np.zeros(n), np.zeros(n)) for p, n in zip(ps, sizes)]
    for step in range(1, 4):
        grads = [rng.normal(size=n).astype(np.float32) for n in sizes]
        for g, gd in zip(grads, dev_g):
            gd.copy_(to_dev(g))
        qg.qg_adam_multi(segs, 0.9, 0.999, 1e-8, step, zero_grad=True)
        ref = [OA.adam_step(pp, g.astype(np.float64), m, v, step, lr) for (pp, m, v), g, lr in zip(ref, grads, lrs)]
        torch.cuda.synchronize()
        for gd in dev_g:
            assert not gd.any().item()
    for dp, (pp, _, _) in zip(dev_p, ref):
        np.testing.assert_allclose(dp.cpu().numpy(), pp, rtol=1e-5, atol=1e-6)
    # the device step counter gives the same updates as the host step count
    dev_p2 = [to_dev(p) for p in ps]
    dev_g2 = [torch.zeros(n, device="cuda") for n in sizes]
    dev_m2 = [torch.zeros(n, device="cuda") for n in sizes]
    dev_v2 = [torch.zeros(n, device="cuda") for n in sizes]
    segs2 = qg.adam_segments(dev_p2, dev_g2, dev_m2, dev_v2, lrs)
    state = torch.zeros(4, dtype=torch.int32, device="cuda")
    rng2 = synth.rng_for(43)
    [rng2.normal(size=n) for n in sizes]
    for step in range(1, 4):
        grads = [rng2.normal(size=n).astype(np.float32) for n in sizes]
        for g, gd in zip(grads, dev_g2):
            gd.copy_(to_dev(g))
        qg.qg_adam_multi(segs2, 0.9, 0.999, 1e-8, 0, zero_grad=True, step_state=state)
    torch.cuda.synchronize()
    assert int(state[0].item()) == 3
    for a, b in zip(dev_p2, dev_p):
        assert torch.equal(a, b)
    # zero_grad off leaves the gradients in place
    for gd in dev_g:
        gd.fill_(1.0)
    qg.qg_adam_multi(segs, 0.9, 0.999, 1e-8, 4, zero_grad=False)
    torch.cuda.synchronize()
    for gd in dev_g:
        assert bool((gd == 1.0).all().item())


@pytest.mark.parametrize("n,tile,deg", [(3001, (16, 16), 3), (40, (8, 8), 3), (5000, (32, 8), 3), (3001, (16, 16), 1),
                                       (777, (16, 16), 0)])
def test_fused_equals_two_call_path(qgm, n, tile, deg):
    """qg_decode_project == qg_decode_residuals + qg_project bit for bit; qg_render_decode_bwd ==
    qg_render_bwd + qg_decode_residuals_bwd, with or without the decoded attributes, up to the order of
    float atomics."""
    qg, raster = qgm
    rng = synth.rng_for(50 + n)
    sc = synth.draw_scene(rng, n, 1.0, -3.5, 0.5)
    cams = cams_small(96, 72)
    prev = to_dev(sc.planes())
    lat = to_dev(rng.normal(0, 1.2, size=(8, n)).astype(np.float32))
    W1 = to_dev((rng.normal(size=(32, 8)) * 0.05).astype(np.float32))
    W2 = to_dev((rng.normal(size=(56, 32)) * 0.02).astype(np.float32))
    lp = to_dev(rng.normal(0, 0.02, size=(3, n)).astype(np.float32))
    a = to_dev(rng.normal(0, 1.0, size=n).astype(np.float32))
    hp = (-0.5, 1.01, 0.3)
    bg = (0.1, 0.2, 0.3)
    # two-call path
    r1 = raster.Rasterizer(n, cams, tile=tile, bg=bg, sh_degree=deg)
    attrs = torch.empty_like(prev)
    qg.qg_decode_residuals(n, n, prev, lat, 8, W1, W2, 32, 56, lp, a, *hp, attrs)
    r1.forward(attrs)
    # fused path
    r2 = raster.Rasterizer(n, cams, tile=tile, bg=bg, capacity=r1.capacity, sh_degree=deg)
    attrs2 = torch.empty_like(prev)
    qg.qg_decode_project(n, n, prev, lat, 8, W1, W2, 32, 56, lp, a, *hp, deg, r2.qcams, r2.tile, r2.dilation, r2.t_proj,
                         attrs2)
    r2.bin()
    r2.render()
    torch.cuda.synchronize()
    assert torch.equal(attrs, attrs2)
    for v in range(len(cams)):
        for k in ("splat", "depth", "rect", "ntiles", "flags"):
            assert torch.equal(r1.proj[v][k], r2.proj[v][k]), k
        assert torch.equal(r1.images[v], r2.images[v])
    G = [to_dev(rng.normal(size=(3, c.height, c.width)).astype(np.float32)) for c in cams]
    lam = 0.01
    names = ("lat", "W1", "W2", "lp", "a")
    g1 = {k: torch.zeros_like(t) for k, t in zip(names, (lat, W1, W2, lp, a))}
    ga1 = torch.zeros_like(prev)
    gabs1 = torch.zeros(n, device="cuda")
    r1.backward(attrs, G, ga1, gabs1)
    wsb = qg.qg_decode_bwd_workspace_size(n, 8, 32, 56)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    qg.qg_decode_residuals_bwd(n, n, lat, 8, W1, W2, 32, 56, lp, a, *hp, ga1, lam, g1["lat"], g1["W1"], g1["W2"],
                               g1["lp"], g1["a"], ws, wsb)
    g2 = {k: torch.zeros_like(t) for k, t in zip(names, (lat, W1, W2, lp, a))}
    gabs2 = torch.zeros(n, device="cuda")
    wsb2 = qg.qg_render_decode_bwd_workspace_size(n, len(cams))
    ws2 = torch.empty(wsb2, dtype=torch.uint8, device="cuda")
    qg.qg_render_decode_bwd(n, n, prev, lat, 8, W1, W2, 32, 56, lp, a, *hp, lam, deg, r2.qcams, r2.tile, r2.dilation,
                            r2.t_proj, r2.vals, r2.ranges, bg, r2.t_tf, r2.t_last, G, g2["lat"], g2["W1"], g2["W2"],
                            g2["lp"], g2["a"], gabs2, None, ws2, wsb2)
    # the adjoint given the decoded attributes of the forward (no second decode) gives the same gradients
    g3 = {k: torch.zeros_like(t) for k, t in zip(names, (lat, W1, W2, lp, a))}
    gabs3 = torch.zeros(n, device="cuda")
    qg.qg_render_decode_bwd(n, n, None, lat, 8, W1, W2, 32, 56, lp, a, *hp, lam, deg, r2.qcams, r2.tile, r2.dilation,
                            r2.t_proj, r2.vals, r2.ranges, bg, r2.t_tf, r2.t_last, G, g3["lat"], g3["W1"], g3["W2"],
                            g3["lp"], g3["a"], gabs3, None, ws2, wsb2, attrs=attrs2)
    torch.cuda.synchronize()
    # the blend adjoint uses float atomics, so equality is up to their summation order
    for k in names:
        assert rel_l2(g2[k].cpu().numpy(), g1[k].cpu().numpy()) <= 1e-5, k
        assert rel_l2(g3[k].cpu().numpy(), g2[k].cpu().numpy()) <= 1e-5, k
    assert rel_l2(gabs2.cpu().numpy(), gabs1.cpu().numpy()) <= 1e-5
    assert rel_l2(gabs3.cpu().numpy(), gabs2.cpu().numpy()) <= 1e-5


@pytest.mark.parametrize("n", [1, 2, 1000, 100003])
def test_gate_init_exact_median_and_logits(qgm, n):
    qg, raster = qgm
    from oracle import gate as OG
    from paper_2412_04469_amd import fit
    rng = synth.rng_for(60 + n)
    x = rng.integers(0, 500, size=n).astype(np.float32)  # exact norms: sqrt(x^2) = x in float32
    x[rng.uniform(size=n) < 0.05] = 0.0
    d = np.stack([x * np.where(rng.uniform(size=n) < 0.5, -1, 1), np.zeros(n, np.float32)]).astype(np.float32)
    a, p, med = fit.gate_init(to_dev(d))
    torch.cuda.synchronize()
    assert med.item() == np.sort(np.abs(x))[(n - 1) // 2]
    p_ref, a_ref = OG.gate_init(d.T.astype(np.float64), -0.5, 1.01, 0.3)
    np.testing.assert_allclose(p.cpu().numpy(), p_ref, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(a.cpu().numpy(), a_ref, rtol=1e-5, atol=1e-3)


def test_viewspace_gradient_difference_parity(qgm):
    """Eq. 9 on the GPU (one adjoint pass per view with image gradient 2 (I_{t-1} - I_t)/(3HW)) against the
    oracle's adjoint; the oracle's one-pass form is itself pinned to the literal two-pass form."""
    qg, raster = qgm
    from oracle import gate as OG
    from paper_2412_04469_amd import fit
    sc = small_scene(seed=14, n=2500)
    moved = sc.copy()
    rng = synth.rng_for(61)
    mv = rng.permutation(sc.n)[:250]
    moved.means[mv] += rng.normal(0, 0.05, size=(250, 3)).astype(np.float32)
    cams = cams_small(112, 84)
    prev64 = sc.planes().astype(np.float64)
    d_ref = np.zeros((sc.n, 2))
    gt_prev, gt_cur = [], []
    for cam in cams:
        rp = OR.render(prev64, cam)
        rc = OR.render(moved.planes().astype(np.float64), cam)
        ip = rp["image"].astype(np.float32)
        ic = rc["image"].astype(np.float32)
        ic[:, ~keep_mask(rp)] = ip[:, ~keep_mask(rp)]  # no gradient where the render's decisions are marginal
        gt_prev.append(ip)
        gt_cur.append(ic)
        planes = torch.tensor(prev64)
        r = OR.render(planes, cam, grad_image=OG.dt_image_gradient(ip, ic))
        d_ref += r["g_xy"]
    d = fit.viewspace_gradient_difference(to_dev(sc.planes()), cams, [to_dev(x) for x in gt_prev],
                                          [to_dev(x) for x in gt_cur])
    torch.cuda.synchronize()
    dg = d.cpu().numpy().T
    assert np.abs(d_ref).max() > 0
    assert rel_l2(dg, d_ref) <= 1e-3
    a, p, med = fit.gate_init(d)
    p_ref, _ = OG.gate_init(d_ref, -0.5, 1.01, 0.3)
    assert rel_l2(p.cpu().numpy(), p_ref) <= 1e-2
