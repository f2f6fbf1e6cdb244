"""Multi-view batching, blend scheduling and graph replay (GPU, through the C ABI).

* Blend scheduling (LDS batch depth 32/64/128, heaviest-first tile order) changes no result: images,
  T_final and last are bit-identical, the adjoint equal up to the order of its float atomics.
* A batched multi-view launch equals the per-view launches: images and T_final bit-identical, each tile's
  entry list identical, each pixel's last contributor at the same position in its tile's list; the
  attribute gradient equals the sum of the per-view gradients up to float atomic order.
* A captured fit step replays to the same result as the same step run eagerly from the same state.
"""
import numpy as np
import pytest
import torch

from _helpers import rel_l2, small_scene, to_dev
from paper_2412_04469_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qgm():
    from paper_2412_04469_amd import qg, raster
    qg.lib()
    return qg, raster


def uneven_cams():
    """Three views of uneven resolution around the scene."""
    return [synth.make_camera((0.0, 0.0, -4.0), 160, 120, f=160),
            synth.make_camera((2.0, -0.5, -3.4), 96, 200, f=110),
            synth.make_camera((-2.5, 0.4, -3.0), 70, 45, f=64)]


def _render(raster, sc, cams, tile=(16, 16), batch=0, heaviest_first=False):
    rast = raster.Rasterizer(sc.n, cams, tile=tile, batch=batch, heaviest_first=heaviest_first, bg=(0.1, 0.2, 0.3))
    attrs = to_dev(sc.planes())
    rast.forward(attrs)
    torch.cuda.synchronize()
    return rast, attrs


def _grad(rast, attrs, gis):
    g = torch.zeros_like(attrs)
    rast.backward(attrs, gis, g)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def _grad_images(cams, seed):
    rng = np.random.default_rng(seed)
    return [to_dev(rng.normal(size=(3, c.height, c.width)) / (3 * c.width * c.height)) for c in cams]


def _xcd_of_tiles(cams, tile):
    """Per global tile, its XCD under the 4x4 super-tile order: the super-tile's index (views in turn, rows of
    super-tiles in turn) mod 8."""
    out, j = [], 0
    for c in cams:
        gw, gh = -(-c.width // tile[0]), -(-c.height // tile[1])
        sw, sh = -(-gw // 4), -(-gh // 4)
        ty, tx = np.divmod(np.arange(gw * gh), gw)
        out.append((j + (ty // 4) * sw + tx // 4) % 8)
        j += sw * sh
    return np.concatenate(out)


@pytest.mark.parametrize("large", [False, True])
def test_schedule_is_heaviest_first_per_xcd(qgm, large):
    """The schedule holds 8 XCD segments: each holds exactly the tiles that the super-tile order puts on that
    XCD, heaviest first (up to the 1/8-octave bucket width, empty tiles last), and together they are a
    permutation of all tiles.  Up to 2^18 tiles one workgroup builds it; above (three 3840x2160 views in 8x8
    tiles: 388,800) a histogram, a scan and a scatter kernel do.  Either way the images equal the unscheduled
    render's bit for bit."""
    qg, raster = qgm
    sc = small_scene(seed=30, n=5000)
    cams = uneven_cams() if not large else [synth.make_camera((0.3 * v, 0.0, -4.0), 3840, 2160, f=3200)
                                            for v in range(3)]
    tile = (16, 16) if not large else (8, 8)
    rast, _ = _render(raster, sc, cams, tile, heaviest_first=True)
    assert (rast.total_tiles > 1 << 18) == large
    s = rast.schedule.cpu().numpy().view(np.uint32).astype(np.int64)
    hdr = 16 + 8 * 512  # QG_SCHEDULE_HEADER_WORDS
    start, length = s[0:8], s[8:16]
    assert start[0] == 0 and np.array_equal(start[1:], np.cumsum(length)[:-1]) and length.sum() == rast.total_tiles
    order = s[hdr:hdr + rast.total_tiles]
    assert np.array_equal(np.sort(order), np.arange(rast.total_tiles))
    xcd = _xcd_of_tiles(cams, tile)
    rg = rast.ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    lens = rg[:, 1] - rg[:, 0]
    for x in range(8):
        seg = order[start[x]:start[x] + length[x]]
        assert np.all(xcd[seg] == x)
        ln = lens[seg]
        if len(ln) == 0:
            continue
        assert ln[0] == ln.max() or ln[0] * 9 > ln.max() * 8  # within one bucket (1/8 octave) of the heaviest
        assert np.all(ln[1:] * 8 <= ln[:-1] * 9 + 8)  # non-increasing up to the bucket width
        if (ln == 0).any():
            assert np.all(ln[int(np.argmax(ln == 0)):] == 0)  # empty tiles last
    ref, _ = _render(raster, sc, cams, tile)
    for v in range(len(cams)):
        assert torch.equal(rast.images[v], ref.images[v])


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_blend_scheduling_does_not_change_results(qgm, tile):
    qg, raster = qgm
    sc = small_scene(seed=31, n=4000)
    cams = uneven_cams()
    ref, attrs = _render(raster, sc, cams, tile)
    gis = _grad_images(cams, 7)
    g_ref = _grad(ref, attrs, gis)
    for batch, heaviest_first in [(32, False), (128, False), (64, True), (128, True), (32, True)]:
        r, _ = _render(raster, sc, cams, tile, batch, heaviest_first)
        for rep in range(2):  # a second launch on the same buffers gives the same result
            if rep:
                r.render()
                torch.cuda.synchronize()
            for v in range(len(cams)):
                assert torch.equal(r.images[v], ref.images[v]), (batch, heaviest_first, v)
                assert torch.equal(r.tfinal[v], ref.tfinal[v])
                assert torch.equal(r.last[v], ref.last[v])
        g = _grad(r, attrs, gis)
        assert rel_l2(g, g_ref) <= 1e-5, (batch, heaviest_first, rel_l2(g, g_ref))


def _tile_of_pixels(cam, tw, th, off):
    gw = -(-cam.width // tw)
    ty = np.arange(cam.height) // th
    tx = np.arange(cam.width) // tw
    return off + ty[:, None] * gw + tx[None, :]


@pytest.mark.parametrize("heaviest_first", [False, True])
def test_batched_views_equal_single_views(qgm, heaviest_first):
    qg, raster = qgm
    sc = small_scene(seed=32, n=6000)
    cams = uneven_cams()
    tw, th = 16, 16
    bat, attrs = _render(raster, sc, cams, (tw, th), 64, heaviest_first)
    gis = _grad_images(cams, 8)
    g_bat = _grad(bat, attrs, gis)
    g_sum = np.zeros_like(g_bat)
    brg = bat.ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    bvals = bat.vals.cpu().numpy().view(np.uint32)
    off = 0
    for v, cam in enumerate(cams):
        one, _ = _render(raster, sc, [cam], (tw, th))
        assert torch.equal(bat.images[v], one.images[0])
        assert torch.equal(bat.tfinal[v], one.tfinal[0])
        org = one.ranges.cpu().numpy().view(np.uint32).astype(np.int64)
        ovals = one.vals.cpu().numpy().view(np.uint32)
        nt = org.shape[0]
        for t in range(nt):  # each tile's entry list is the same Gaussians in the same order
            a = bvals[brg[off + t, 0]:brg[off + t, 1]]
            b = ovals[org[t, 0]:org[t, 1]]
            assert np.array_equal(a, b), (v, t)
        tb = _tile_of_pixels(cam, tw, th, off)
        to = _tile_of_pixels(cam, tw, th, 0)
        pos_b = bat.last[v].cpu().numpy().view(np.uint32).astype(np.int64) - brg[tb, 0]
        pos_o = one.last[0].cpu().numpy().view(np.uint32).astype(np.int64) - org[to, 0]
        assert np.array_equal(pos_b, pos_o)
        g_sum += _grad(one, attrs, [gis[v]])
        off += nt
    assert off == bat.total_tiles
    assert rel_l2(g_bat, g_sum) <= 1e-5


def _fit_inputs(n=3000, seed=33):
    from paper_2412_04469_amd.fit import FitConfig, render_views
    base = small_scene(seed=seed, n=n)
    rng = synth.rng_for(seed + 1)
    moved = base.copy()
    moved.means[: n // 10] += rng.normal(0, 0.05, size=(n // 10, 3)).astype(np.float32)
    cams = uneven_cams()
    prev = to_dev(base.planes())
    gts = render_views(to_dev(moved.planes()), cams, FitConfig())
    return prev, cams, gts


def _state(f):
    keys = ["lat", "lp", "a", "W1", "W2"]
    return ([f.params[k].clone() for k in keys], [f.m[k].clone() for k in keys], [f.v[k].clone() for k in keys],
            f.step_state.clone())


def _restore(f, st):
    keys = ["lat", "lp", "a", "W1", "W2"]
    p, m, v, s = st
    for k, a, b, c in zip(keys, p, m, v):
        f.params[k].copy_(a)
        f.m[k].copy_(b)
        f.v[k].copy_(c)
        f.grads[k].zero_()
    f.step_state.copy_(s)


def test_graph_replay_matches_eager_step(qgm):
    qg, raster = qgm
    from paper_2412_04469_amd.fit import BatchedFitter
    prev, cams, gts = _fit_inputs()
    f = BatchedFitter(prev, cams, gts, heaviest_first=True, graph=True)
    f.size_capacity()
    f.step()  # eager first step, then capture
    torch.cuda.synchronize()
    assert f.graphs[0] is not None
    keys = ["lat", "lp", "a", "W1", "W2"]
    for rnd in range(3):
        s0 = _state(f)
        f._enqueue(0)  # the same step, eagerly
        torch.cuda.synchronize()
        eager_imgs = [im.clone() for im in f.rasts[0].images]
        eager = _state(f)
        _restore(f, s0)
        f.step()  # graph replay
        torch.cuda.synchronize()
        assert not f.overflowed()
        for a, b in zip(f.rasts[0].images, eager_imgs):
            assert torch.equal(a, b), rnd
        rep = _state(f)
        assert torch.equal(rep[3], eager[3])  # device step counter advanced once
        for k, p0, pe, pr in zip(keys, s0[0], eager[0], rep[0]):
            de, dr = (pe - p0).cpu().numpy(), (pr - p0).cpu().numpy()
            assert rel_l2(dr, de) <= 1e-3, (rnd, k, rel_l2(dr, de))
    assert int(f.step_state[0].item()) == 1 + 3


def test_batched_fit_reduces_loss(qgm):
    qg, raster = qgm
    from paper_2412_04469_amd.fit import BatchedFitter
    prev, cams, gts = _fit_inputs(seed=35)
    f = BatchedFitter(prev, cams, gts, heaviest_first=True, graph=True)
    f.size_capacity()
    f.step()
    first = np.mean(f.losses())
    for _ in range(30):
        f.step()
    assert not f.overflowed()
    last = np.mean(f.losses())
    assert last < first, (first, last)


def test_frame_fitter_graph_replay_matches_eager_step(qgm):
    """The per-view graphs of FrameFitter(graph=True): a replayed step of view v equals the same step run
    eagerly from the same state (image bit for bit, parameter updates up to float atomic order), for each view
    and again after other views' replays; the device step counter advances once per step."""
    qg, raster = qgm
    from paper_2412_04469_amd.fit import FitConfig, FrameFitter, render_views
    n = 3000
    base = small_scene(seed=36, n=n)
    rng = synth.rng_for(37)
    moved = base.copy()
    moved.means[: n // 10] += rng.normal(0, 0.05, size=(n // 10, 3)).astype(np.float32)
    cams = [synth.make_camera((0.0, 0.0, -4.0), 160, 120, f=160),
            synth.make_camera((1.5, -0.3, -3.6), 160, 120, f=150),
            synth.make_camera((-1.8, 0.4, -3.2), 160, 120, f=140)]
    gts = render_views(to_dev(moved.planes()), cams, FitConfig())
    f = FrameFitter(to_dev(base.planes()), cams, gts, FitConfig(), graph=True)
    f.size_capacity()
    for v in range(len(cams)):  # first step of each view: eager, then captured
        f.step(v)
    torch.cuda.synchronize()
    assert sorted(f.graphs) == [0, 1, 2]
    keys = ["lat", "lp", "a", "W1", "W2"]
    for rnd, v in enumerate([0, 1, 2, 1]):
        s0 = _state(f)
        f.step(v, eager=True)
        torch.cuda.synchronize()
        eager_img = f.rast.images[0].clone()
        eager = _state(f)
        _restore(f, s0)
        f.step(v)  # graph replay
        torch.cuda.synchronize()
        assert not f.rast.overflowed()
        assert torch.equal(f.rast.images[0], eager_img), rnd
        rep = _state(f)
        assert torch.equal(rep[3], eager[3])
        for k, p0, pe, pr in zip(keys, s0[0], eager[0], rep[0]):
            de, dr = (pe - p0).cpu().numpy(), (pr - p0).cpu().numpy()
            assert rel_l2(dr, de) <= 1e-3, (rnd, k, rel_l2(dr, de))
    assert int(f.step_state[0].item()) == len(cams) + 4


@pytest.mark.parametrize("heaviest_first", [False, True])
def test_render_fwd_l1_equals_render_then_l1(qgm, heaviest_first):
    """qg_render_fwd_l1 over three uneven views equals qg_render_fwd followed by one qg_l1_loss per view: image,
    T_final and last bit for bit, the L1 gradient bit for bit (per-view scale), and each view's L1 and MSE from
    its tiles' partials (qg_loss_reduce_parts) equal to qg_loss_reduce's within rounding."""
    qg, raster = qgm
    sc = small_scene(seed=38, n=5000)
    cams = uneven_cams()
    ref, attrs = _render(raster, sc, cams, (16, 16), 64, heaviest_first)
    rng = np.random.default_rng(39)
    gts = [to_dev(rng.uniform(0.0, 1.0, size=(3, c.height, c.width))) for c in cams]
    scales = [1.0, 0.5, 2.0]
    ref_grads, ref_loss = [], []
    for v, c in enumerate(cams):
        cnt = 3 * c.width * c.height
        g = torch.empty_like(gts[v])
        part = torch.empty(2 * qg.qg_loss_blocks(cnt), dtype=torch.float64, device="cuda")
        out = torch.zeros(2, dtype=torch.float64, device="cuda")
        qg.qg_l1_loss(cnt, ref.images[v], gts[v], scales[v], g, part)
        qg.qg_loss_reduce(cnt, part, out)
        ref_grads.append(g)
        ref_loss.append(out.cpu().numpy())
    fused = raster.Rasterizer(sc.n, cams, tile=(16, 16), batch=64, heaviest_first=heaviest_first,
                              bg=(0.1, 0.2, 0.3))
    fused.forward(attrs)  # binning (and a plain render, overwritten next)
    grads = [torch.full_like(g, 7.0) for g in gts]
    part = torch.full((2 * fused.total_tiles,), -1.0, dtype=torch.float64, device="cuda")
    fused.render_l1(gts, scales, grads, part)
    torch.cuda.synchronize()
    first = 0
    for v, c in enumerate(cams):
        assert torch.equal(fused.images[v], ref.images[v])
        assert torch.equal(fused.tfinal[v], ref.tfinal[v])
        assert torch.equal(fused.last[v], ref.last[v])
        assert torch.equal(grads[v], ref_grads[v]), v
        nt = qg.qg_total_tiles([c], fused.tile)
        out = torch.zeros(2, dtype=torch.float64, device="cuda")
        qg.qg_loss_reduce_parts(nt, 3 * c.width * c.height, part[2 * first:], out)
        got = out.cpu().numpy()
        assert np.allclose(got, ref_loss[v], rtol=1e-6, atol=0), (v, got, ref_loss[v])
        first += nt
    assert first == fused.total_tiles
    assert (part.cpu().numpy() >= 0).all()  # every tile wrote its partials
