"""Pins of the masked-training oracle (Sec. 3.3 "Adaptive Masked Training"): closed forms and invariants."""
import math

import numpy as np

from oracle import composite as C
from oracle import loss as L
from oracle import mask as M


def test_dilate_single_pixel_is_offset_square():
    """k = 48: one set pixel at (x0, y0) sets exactly x in [x0 - 23, x0 + 24], y in [y0 - 23, y0 + 24]
    (the window of (x, y) is x + [-24, 23]); clipped at the image border."""
    H, W = 80, 100
    for (x0, y0) in [(50, 40), (0, 0), (99, 79), (10, 70)]:
        m = np.zeros((H, W), bool)
        m[y0, x0] = True
        d = M.dilate(m, 48)
        X, Y = np.meshgrid(np.arange(W), np.arange(H))
        want = (X >= x0 - 23) & (X <= x0 + 24) & (Y >= y0 - 23) & (Y <= y0 + 24)
        assert np.array_equal(d, want), (x0, y0)


def test_dilate_odd_kernel_is_centred():
    H, W = 20, 30
    m = np.zeros((H, W), bool)
    m[7, 11] = True
    d = M.dilate(m, 5)
    assert d.sum() == 25 and d[5:10, 9:14].all()
    assert np.array_equal(M.dilate(m, 1), m)


def test_dilate_distributes_over_union_and_limits():
    rng = np.random.default_rng(0)
    H, W = 48, 64
    a = rng.random((H, W)) < 0.01
    b = rng.random((H, W)) < 0.01
    assert np.array_equal(M.dilate(a | b, 48), M.dilate(a, 48) | M.dilate(b, 48))
    assert not M.dilate(np.zeros((H, W), bool), 48).any()
    assert M.dilate(np.ones((H, W), bool), 48).all()


def test_tile_flags_of_one_dilated_pixel():
    """The tiles touched by the 48 x 48 square of one pixel, with ragged edge tiles (100 x 80 at 16 x 16)."""
    H, W = 80, 100
    m = np.zeros((H, W), bool)
    m[30, 60] = True
    f = M.tile_flags(M.dilate(m, 48), 16, 16)
    gw = -(-W // 16)
    x0, x1, y0, y1 = 60 - 23, min(W - 1, 60 + 24), 30 - 23, min(H - 1, 30 + 24)
    want = np.zeros_like(f)
    for ty in range(y0 // 16, y1 // 16 + 1):
        for tx in range(x0 // 16, x1 // 16 + 1):
            want[ty * gw + tx] = True
    assert np.array_equal(f, want)


def test_masked_l1_closed_forms():
    rng = np.random.default_rng(1)
    r = rng.random((3, 12, 10))
    g = rng.random((3, 12, 10))
    full, gfull = L.l1(r, g)
    lm, gm = M.masked_l1(r, g, np.ones((12, 10), bool))
    assert lm == full and np.array_equal(gm, gfull)
    l0, g0 = M.masked_l1(r, g, np.zeros((12, 10), bool))
    assert l0 == 0.0 and not g0.any()
    # constant difference c on a mask of m pixels: loss = c * 3m / (3HW), gradient sign / (3HW) there
    c = 0.25
    pm = np.zeros((12, 10), bool)
    pm[2:5, 3:9] = True
    lc, gc = M.masked_l1(g + c, g, pm)
    assert math.isclose(lc, c * pm.sum() / 120.0, rel_tol=1e-12)
    assert np.allclose(gc[:, pm], 1.0 / 360.0) and not gc[:, ~pm].any()


def _splats(xy, conic, op, depth):
    n = len(op)
    return {"xy": np.asarray(xy, float), "conic": np.asarray(conic, float), "opacity": np.asarray(op, float),
            "rgb": np.full((n, 3), 0.5), "depth": np.asarray(depth, float)}


def test_dynamic_mask_is_union_of_footprints():
    """The dynamic-only render reaches exactly the union of the dynamic splats' alpha >= 1/255 ellipses, even
    where one dynamic splat lies behind another nearly opaque one (the first splat leaves T >= 0.01)."""
    W, H = 48, 40
    xy = [[20.3, 18.7], [22.0, 20.0], [5.5, 33.1]]
    conic = [[0.05, 0.01, 0.08], [0.02, -0.005, 0.03], [0.3, 0.0, 0.2]]
    op = [0.999, 0.6, 0.3]
    dep = [1.0, 2.0, 3.0]
    r = C.composite_image(_splats(xy, conic, op, dep), W, H)
    want = np.zeros((H, W), bool)
    for k in range(3):
        want |= M.footprint(xy[k], conic[k], op[k], W, H)
    assert np.array_equal(M.dynamic_mask(r["t_final"]), want)
    assert want.sum() > 100 and not want.all()


def test_single_dynamic_splat_footprint_count():
    """Isotropic sigma' = 4 px, o = 0.5, centred on a pixel centre: 489 pixel centres within radius
    4 sqrt(2 ln 127.5)."""
    fp = M.footprint([20.5, 20.5], [1 / 16, 0.0, 1 / 16], 0.5, 41, 41)
    assert fp.sum() == 489


def test_dynamic_flags_threshold_is_strict_on_the_view_mean():
    V, t = 4, 1e-3
    # a 2 x 2 image makes the NDC factor 1: norms 5e-3 / 4 > 1e-3; 4e-3 / 4 == 1e-3 is not dynamic; 0 is static
    d = np.array([[3e-3, 0.0, 0.0, -2.4e-3], [4e-3, 4e-3, 0.0, 3.2e-3]])
    assert list(M.dynamic_flags(d, V, 2, 2, t)) == [True, False, False, False]
    assert list(M.dynamic_flags(d, 1, 2, 2, t)) == [True, True, False, True]


def test_dynamic_flags_use_ndc_units_per_axis():
    """A 1-pixel gradient is 2/W (x) or 2/H (y) in NDC: at W = 4, H = 2 the x component counts twice."""
    d = np.array([[1e-3, 0.0], [0.0, 1e-3]])
    assert list(M.dynamic_flags(d, 1, 4, 2, 1e-3)) == [True, False]
    assert list(M.dynamic_flags(d, 1, 1352, 1014, 0.6)) == [True, False]  # 0.676 and 0.507


def test_masked_iterations():
    assert M.masked_iterations(100, 0.30) == 30
    assert M.masked_iterations(100, 0.65) == 65
    assert M.masked_iterations(7, 0.30) == 3
    assert M.masked_iterations(10, 0.0) == 0
