"""Pins of the D-SSIM oracle (Eq. 3's D-SSIM term): closed forms, invariants and finite differences."""
import math

import numpy as np

from oracle import ssim as S


def test_window_is_normalised_separable_gaussian():
    g = S.window_1d()
    assert len(g) == 11 and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1])
    assert math.isclose(g[6] / g[5], math.exp(-1.0 / (2 * 1.5 ** 2)), rel_tol=1e-14)
    w = S.window_2d()
    assert abs(w.sum() - 1.0) < 1e-14 and np.allclose(w, np.outer(g, g))


def test_identical_images_give_one():
    rng = np.random.default_rng(0)
    x = rng.random((3, 20, 24))
    m = S.ssim_map(x, x).numpy()
    assert np.allclose(m, 1.0, atol=1e-12)
    loss, grad = S.dssim(x, x)
    assert abs(loss) < 1e-12 and np.abs(grad).max() < 1e-10


def test_symmetric_in_its_arguments():
    rng = np.random.default_rng(1)
    x, y = rng.random((2, 3, 17, 19))
    assert np.allclose(S.ssim_map(x, y).numpy(), S.ssim_map(y, x).numpy(), atol=1e-14)


def test_constant_images_closed_form_in_the_interior():
    """x = a, y = b everywhere: away from the zero-padded border mu = a, b and every variance is 0, so
    SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.7, 0.2
    x = np.full((1, 30, 30), a)
    y = np.full((1, 30, 30), b)
    m = S.ssim_map(x, y).numpy()[0]
    want = (2 * a * b + S.C1) / (a * a + b * b + S.C1)
    assert np.allclose(m[5:25, 5:25], want, atol=1e-13)
    assert abs(m[0, 0] - want) > 1e-3  # the border sees the zero padding


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    x = rng.random((3, 14, 15))
    y = rng.random((3, 14, 15))
    _, g = S.dssim(x, y)
    h = 1e-6
    for (c, i, j) in [(0, 0, 0), (1, 7, 7), (2, 13, 14), (0, 3, 11), (2, 10, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (S.dssim(xp, y, False)[0] - S.dssim(xm, y, False)[0]) / (2 * h)
        assert abs(fd - g[c, i, j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (c, i, j, fd, g[c, i, j])


def test_eq3_mix():
    rng = np.random.default_rng(3)
    x, y = rng.random((2, 3, 12, 13))
    l, g = S.loss_eq3(x, y, 0.2)
    l1 = np.abs(x - y).mean()
    ds, gds = S.dssim(x, y)
    assert math.isclose(l, 0.8 * l1 + 0.2 * ds, rel_tol=1e-14)
    assert np.allclose(g, 0.8 * np.sign(x - y) / x.size + 0.2 * gds)
