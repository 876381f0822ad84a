"""Pins of the FP64 loss oracle ((1 - lambda) L2 + lambda D-SSIM, Sec. 3.2) against facts fixed
by the mathematics: the window against scipy's Gaussian window, SSIM of an image with itself,
closed forms of the local statistics of constant planes (which also fix the zero padding at the
border) and of linear ramps (which fix the variance and covariance terms and C2), the pure L2
case, and central finite differences for the gradient.
"""
import numpy as np
import pytest
from scipy.signal import windows

from oracle import loss as OL

C1, C2 = 0.01 ** 2, 0.03 ** 2


def _g1():
    g = windows.gaussian(11, 1.5)
    return g / g.sum()


def test_window_is_scipy_gaussian():
    w = OL.window()
    assert w.shape == (11, 11)
    np.testing.assert_allclose(w, np.outer(_g1(), _g1()), rtol=1e-14, atol=0)
    assert abs(w.sum() - 1.0) < 1e-14


def test_ssim_of_image_with_itself_is_one():
    x = np.random.default_rng(1).uniform(0, 1, (2, 9, 14))
    np.testing.assert_allclose(OL.ssim_map(x, x), 1.0, rtol=0, atol=1e-12)
    assert OL.loss(x, x) == pytest.approx(0.0, abs=1e-12)


def test_constant_planes_closed_form_with_border():
    """x = a, y = b everywhere. At pixel (i, j) the window mass inside the image is
    m = G(i) G(j), G the 1D partial sums of the window; then mu_x = a m, E[x^2] = a^2 m,
    var_x = a^2 m (1 - m), cov = a b m (1 - m), and SSIM follows from its definition."""
    h, w_ = 17, 22
    a, b = 0.7, 0.3
    x = np.full((1, h, w_), a)
    y = np.full((1, h, w_), b)
    g = _g1()

    def mass(n):
        out = np.zeros(n)
        for i in range(n):
            for k in range(-5, 6):
                if 0 <= i + k < n:
                    out[i] += g[k + 5]
        return out

    m = np.outer(mass(h), mass(w_))
    s2 = a * a + b * b
    want = ((2 * a * b * m * m + C1) * (2 * a * b * m * (1 - m) + C2)) / \
        ((s2 * m * m + C1) * (s2 * m * (1 - m) + C2))
    np.testing.assert_allclose(OL.ssim_map(x, y)[0], want, rtol=1e-12, atol=1e-14)
    # interior: the textbook luminance term alone
    assert OL.ssim_map(x, y)[0, 8, 11] == pytest.approx((2 * a * b + C1) / (s2 + C1), rel=1e-12)


def test_linear_ramps_closed_form_interior():
    """x = al i + be j + c0, y = ga i + de j + c1. The window is symmetric and separable, so at
    interior pixels the local mean is the value itself, var_x = (al^2 + be^2) v and
    cov = (al ga + be de) v, with v = sum_k g_k k^2 the 1D window's second moment."""
    h, w_ = 21, 24
    al, be, c0 = 0.013, -0.021, 0.45
    ga, de, c1 = -0.017, 0.009, 0.55
    i, j = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w_, dtype=np.float64), indexing="ij")
    x = (al * i + be * j + c0)[None]
    y = (ga * i + de * j + c1)[None]
    g = _g1()
    v = float(np.sum(g * (np.arange(11) - 5.0) ** 2))
    mx, my = x[0], y[0]
    vx, vy, cxy = (al * al + be * be) * v, (ga * ga + de * de) * v, (al * ga + be * de) * v
    want = ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    got = OL.ssim_map(x, y)[0]
    np.testing.assert_allclose(got[5:-5, 5:-5], want[5:-5, 5:-5], rtol=1e-11)
    # the covariance is negative here, so the structure term is below one
    assert np.all(got[5:-5, 5:-5] < 0.999)


def test_pure_l2_case():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(0, 1, (3, 8, 10)), rng.uniform(0, 1, (3, 8, 10))
    n = 1000
    assert OL.loss(x, y, lam=0.0, n=n) == pytest.approx(np.sum((x - y) ** 2) / n, rel=1e-14)
    np.testing.assert_allclose(OL.loss_grad(x, y, lam=0.0, n=n), 2 * (x - y) / n, rtol=1e-14, atol=0)


def test_gradient_vanishes_at_identity():
    x = np.random.default_rng(4).uniform(0, 1, (2, 12, 13))
    assert np.max(np.abs(OL.loss_grad(x, x))) < 1e-15


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_gradient_finite_differences(lam):
    rng = np.random.default_rng(5)
    x, y = rng.uniform(0, 1, (2, 12, 15)), rng.uniform(0, 1, (2, 12, 15))
    g = OL.loss_grad(x, y, lam=lam)
    eps = 1e-6
    for idx in [(0, 0, 0), (0, 11, 14), (1, 0, 14), (1, 6, 7), (0, 3, 1), (1, 10, 5), (0, 5, 12)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (OL.loss(xp, y, lam) - OL.loss(xm, y, lam)) / (2 * eps)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-13), idx


def test_views_compose_by_element_count():
    """A batch is the sum of its views' terms divided by the batch's element count."""
    rng = np.random.default_rng(6)
    a = (rng.uniform(0, 1, (3, 7, 9)), rng.uniform(0, 1, (3, 7, 9)))
    b = (rng.uniform(0, 1, (3, 11, 5)), rng.uniform(0, 1, (3, 11, 5)))
    n = a[0].size + b[0].size
    both = OL.loss(*a, n=n) + OL.loss(*b, n=n)
    la, lb = OL.loss(*a), OL.loss(*b)
    assert both == pytest.approx((la * a[0].size + lb * b[0].size) / n, rel=1e-13)
