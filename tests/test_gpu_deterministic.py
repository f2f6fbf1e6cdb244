"""Deterministic mode of the adjoints (QG_DETERMINISTIC=1 / qg_set_deterministic): the blend adjoint's per-pair
partials summed in a fixed order, and the fused adjoint's per-chunk weight-gradient rows.  Two runs must give the
same bits, and the result must match the default (float-atomic) mode up to rounding order."""
import numpy as np
import pytest
import torch

from _helpers import cams_small, rel_l2, small_scene, to_dev
from paper_2412_04469_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture
def qgm():
    from paper_2412_04469_amd import qg, raster
    qg.lib()
    qg.qg_set_deterministic(False)
    yield qg, raster
    qg.qg_set_deterministic(False)


def _grads_render_bwd(qg, raster, attrs, cams, G, tile, det):
    qg.qg_set_deterministic(det)
    n = attrs.shape[1]
    r = raster.Rasterizer(n, cams, tile=tile, bg=(0.1, 0.2, 0.3))
    r.forward(attrs)
    out = []
    for _ in range(2):
        ga = torch.zeros_like(attrs)
        gabs = torch.zeros(n, device="cuda")
        gxy = [torch.zeros(2, n, device="cuda") for _ in cams]
        r.backward(attrs, G, ga, gabs, gxy)
        torch.cuda.synchronize()
        out.append((ga, gabs, gxy))
    return out


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_render_bwd_deterministic_runs_are_bitwise_equal(qgm, tile):
    qg, raster = qgm
    sc = small_scene(seed=61, n=4000, ls_mu=-3.0)
    cams = cams_small(144, 104)
    attrs = to_dev(sc.planes())
    rng = synth.rng_for(62)
    G = [to_dev(rng.normal(size=(3, c.height, c.width)).astype(np.float32)) for c in cams]
    atom = _grads_render_bwd(qg, raster, attrs, cams, G, tile, False)
    det = _grads_render_bwd(qg, raster, attrs, cams, G, tile, True)
    (a1, b1, x1), (a2, b2, x2) = det
    assert torch.equal(a1, a2) and torch.equal(b1, b2)
    assert all(torch.equal(u, w) for u, w in zip(x1, x2))
    ga_atom = atom[0][0].cpu().numpy()
    ga_det = a1.cpu().numpy()
    assert rel_l2(ga_det, ga_atom) <= 1e-6
    for lo, hi in ((0, 3), (3, 7), (7, 10), (10, 11), (11, 59)):  # means, quats, log-scales, logits, SH
        assert rel_l2(ga_det[lo:hi], ga_atom[lo:hi]) <= 1e-5, (lo, hi)
    assert rel_l2(b1.cpu().numpy(), atom[0][1].cpu().numpy()) <= 1e-5
    print(f"deterministic vs atomic: rel-L2 {rel_l2(ga_det, ga_atom):.2e}")


def test_fused_adjoint_deterministic(qgm):
    qg, raster = qgm
    n = 3000
    rng = synth.rng_for(63)
    sc = synth.draw_scene(rng, n, 1.0, -3.5, 0.5)
    cams = cams_small(112, 80)
    prev = to_dev(sc.planes())
    lat = to_dev(rng.normal(0, 1.2, size=(8, n)).astype(np.float32))
    W1 = to_dev((rng.normal(size=(32, 8)) * 0.05).astype(np.float32))
    W2 = to_dev((rng.normal(size=(56, 32)) * 0.02).astype(np.float32))
    lp = to_dev(rng.normal(0, 0.02, size=(3, n)).astype(np.float32))
    a = to_dev(rng.normal(0, 1.0, size=n).astype(np.float32))
    hp = (-0.5, 1.01, 0.3)
    bg = (0.1, 0.2, 0.3)
    G = [to_dev(rng.normal(size=(3, c.height, c.width)).astype(np.float32)) for c in cams]
    names = ("lat", "W1", "W2", "lp", "a")

    def run(det):
        qg.qg_set_deterministic(det)
        r = raster.Rasterizer(n, cams, bg=bg)
        attrs = torch.empty_like(prev)
        qg.qg_decode_project(n, n, prev, lat, 8, W1, W2, 32, 56, lp, a, *hp, 3, r.qcams, r.tile, r.dilation, r.t_proj,
                             attrs)
        r.bin()
        assert not r.overflowed()
        r.render()
        wsb = qg.qg_render_decode_bwd_workspace_size(n, len(cams)) + r.det_ws_bytes()
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        outs = []
        for _ in range(2):
            g = {k: torch.zeros_like(t) for k, t in zip(names, (lat, W1, W2, lp, a))}
            gabs = torch.zeros(n, device="cuda")
            qg.qg_render_decode_bwd(n, n, None, lat, 8, W1, W2, 32, 56, lp, a, *hp, 0.01, 3, r.qcams, r.tile,
                                    r.dilation, r.t_proj, r.vals, r.ranges, bg, r.t_tf, r.t_last, G, g["lat"],
                                    g["W1"], g["W2"], g["lp"], g["a"], gabs, None, ws, wsb, attrs=attrs)
            torch.cuda.synchronize()
            outs.append((g, gabs))
        return outs

    atom = run(False)
    det = run(True)
    (d1, b1), (d2, b2) = det
    for k in names:
        assert torch.equal(d1[k], d2[k]), k
        assert rel_l2(d1[k].cpu().numpy(), atom[0][0][k].cpu().numpy()) <= 1e-5, k
    assert torch.equal(b1, b2)


def test_deterministic_mode_needs_room_in_the_workspace(qgm):
    qg, raster = qgm
    sc = small_scene(seed=64, n=500)
    cams = cams_small(64, 48)
    attrs = to_dev(sc.planes())
    r = raster.Rasterizer(500, cams)
    r.forward(attrs)
    qg.qg_set_deterministic(True)
    ga = torch.zeros_like(attrs)
    G = [torch.zeros(3, c.height, c.width, device="cuda") for c in cams]
    with pytest.raises(qg.QGError) as e:  # a workspace sized with the mode off
        qg.qg_render_bwd(500, 500, attrs, 3, r.qcams, r.tile, r.dilation, r.t_proj, r.vals, r.ranges, r.bg, r.t_tf,
                         r.t_last, G, ga, None, None, r.bwd_ws, qg.qg_render_bwd_workspace_size(500, 2))
    assert "deterministic" in str(e.value)
