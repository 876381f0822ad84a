"""Pins of the FP64 oracle against facts fixed by the mathematics, not by the oracle itself.

Each test names what it pins: closed forms of the EWA footprint (Sec. 3.2), library routines
(scipy's spherical harmonics and rotations), invariants of front-to-back compositing
(eq. render-gs), properties of the max-based importance score (eq. importance-score, Sec. 3.3)
and of the per-cluster lists (eq. importance-score-vis), and central finite differences for the
analytic gradient.
"""
import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial.transform import Rotation

import oracle
import scenes
from oracle import F

P = scenes.Params()


def _one(mean, scale, quat, opac, rgb=None, sh=None, deg=0):
    """Scene from per-Gaussian rows (lists)."""
    mean = np.asarray(mean, np.float32).reshape(-1, 3).T
    n = mean.shape[1]
    if sh is None:
        rgb = np.asarray(rgb if rgb is not None else [[1.0, 1.0, 1.0]] * n, np.float64).reshape(-1, 3).T
        sh = (rgb - 0.5) * 2.0 * np.sqrt(np.pi)
    return scenes.Scene(np.ascontiguousarray(mean), np.asarray(scale, np.float32).reshape(-1, 3).T.copy(),
                        np.asarray(quat, np.float32).reshape(-1, 4).T.copy(), np.asarray(opac, np.float32).reshape(-1),
                        np.asarray(sh, np.float32).reshape(-1, n).copy(), deg)


# ----------------------------------------------------------------------------------------------
# Spherical harmonics: orthonormality by exact quadrature, and scipy's complex Y_l^m.
# ----------------------------------------------------------------------------------------------

def _sphere_quadrature(nz=8, nphi=16):
    z, wz = np.polynomial.legendre.leggauss(nz)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    Z, PHI = np.meshgrid(z, phi, indexing="ij")
    r = np.sqrt(1 - Z ** 2)
    dirs = np.stack([r * np.cos(PHI), r * np.sin(PHI), Z], -1).reshape(-1, 3)
    w = (wz[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    return dirs, w


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in z (8 nodes, exact to degree 15) x uniform phi (16 nodes): exact for
    # products of two degree-3 harmonics, so int Y_i Y_j = delta_ij up to rounding.
    dirs, w = _sphere_quadrature()
    Y = oracle.sh_basis(3, dirs)
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def _scipy_real_sh(l, m, d):
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Yc = sps.sph_harm_y(l, abs(m), theta, phi)  # includes the Condon-Shortley phase
    if m > 0:
        return np.sqrt(2) * Yc.real
    if m < 0:
        return np.sqrt(2) * Yc.imag
    return Yc.real


def test_sh_matches_scipy():
    rng = np.random.default_rng(5)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle.sh_basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _scipy_real_sh(l, m, d)
            assert np.abs(Y[:, l * l + l + m] - ref).max() < 1e-12, (l, m)


def test_sh_gradient_tangential_vs_scipy_fd():
    # tangential derivative along a great circle, differenced on scipy's values
    rng = np.random.default_rng(6)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    e = rng.standard_normal((50, 3))
    e -= (e * d).sum(1, keepdims=True) * d
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    h = 1e-5
    dp = np.cos(h) * d + np.sin(h) * e
    dm = np.cos(h) * d - np.sin(h) * e
    G = oracle.sh_basis_grad(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            fd = (_scipy_real_sh(l, m, dp) - _scipy_real_sh(l, m, dm)) / (2 * h)
            an = (G[:, k, :] * e).sum(1)
            assert np.abs(fd - an).max() < 1e-7, (l, m)


# ----------------------------------------------------------------------------------------------
# EWA projection (Sec. 3.2): closed forms and the linearised perspective map.
# ----------------------------------------------------------------------------------------------

def test_projection_closed_form_axis_aligned():
    # R = I camera at (0,0,-4), f = 100; Gaussian at camera-space (x0, 0, z0) with
    # Sigma = diag(a, b, c): Sigma'_xx = (f/z0)^2 a + (f x0/z0^2)^2 c + 0.3,
    # Sigma'_yy = (f/z0)^2 b + 0.3, Sigma'_xy = 0, mean at (f x0/z0 + cx, cy).
    cam = scenes.plain_view()
    x0, wz = 0.25, 0.5
    z0 = wz + 4.0
    s = np.float32([0.05, 0.02, 0.07])
    sc = _one([x0, 0.0, wz], s, [1, 0, 0, 0], [0.8])
    pr = oracle.project(sc, cam, P)[0]
    a, b, c = (np.float64(s) ** 2)
    f = 100.0
    x0d = np.float64(np.float32(x0))
    sxx = (f / z0) ** 2 * a + (f * x0d / z0 ** 2) ** 2 * c + np.float64(np.float32(0.3))
    syy = (f / z0) ** 2 * b + np.float64(np.float32(0.3))
    assert pr[F["vis"]] == 1
    assert abs(pr[F["u"]] - (f * x0d / z0 + 64.0)) < 1e-12
    assert abs(pr[F["v"]] - 48.0) < 1e-12
    assert abs(pr[F["sxx"]] - sxx) < 1e-12 * sxx
    assert abs(pr[F["syy"]] - syy) < 1e-12 * syy
    assert abs(pr[F["sxy"]]) < 1e-15
    assert abs(pr[F["ca"]] - 1 / sxx) < 1e-12 / sxx and abs(pr[F["cc"]] - 1 / syy) < 1e-12 / syy
    # opacity 0.8 > alpha_min * e^4.5, so the support radius is kappa^2
    assert pr[F["qmax"]] == 9.0
    # the rendered image of this single Gaussian is alpha * colour with alpha from the closed form
    out = oracle.render(sc, cam, P)
    px, py = np.meshgrid(np.arange(128) + 0.5, np.arange(96) + 0.5)
    dx, dy = px - pr[F["u"]], py - 48.0
    q = dx ** 2 / sxx + dy ** 2 / syy
    alpha = np.where(q <= 9.0, np.float64(np.float32(0.8)) * np.exp(-0.5 * q), 0.0)
    safe = np.abs(q - 9.0) > 1e-9
    col = out["rgb"][0]
    colour = np.float64(np.float32((1.0 - 0.5) * 2 * np.sqrt(np.pi))) * 0.5 / np.sqrt(np.pi) + 0.5
    assert np.abs(col - alpha * colour)[safe].max() < 1e-12
    assert np.abs(out["T"] - (1 - alpha))[safe].max() < 1e-12
    assert (alpha > 0).sum() > 20


def test_projection_rotation_about_optical_axis():
    # 90 degrees about z swaps the x and y variances; 180 degrees leaves Sigma unchanged
    cam = scenes.plain_view()
    s = [0.05, 0.02, 0.07]
    base = oracle.project(_one([0, 0, 0], s, [1, 0, 0, 0], [0.9]), cam, P)[0]
    r90 = oracle.project(_one([0, 0, 0], s, [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)], [0.9]), cam, P)[0]
    r180 = oracle.project(_one([0, 0, 0], s, [0, 0, 0, 1], [0.9]), cam, P)[0]
    assert abs(r90[F["sxx"]] - base[F["syy"]]) < 1e-6 * base[F["syy"]]
    assert abs(r90[F["syy"]] - base[F["sxx"]]) < 1e-6 * base[F["sxx"]]
    assert abs(r180[F["sxx"]] - base[F["sxx"]]) < 1e-12 * base[F["sxx"]]
    assert abs(r180[F["syy"]] - base[F["syy"]]) < 1e-12 * base[F["syy"]]


def test_projection_matches_linearised_perspective_with_scipy_rotation():
    # Sigma' - lowpass I = Jpi (R Sigma R^T) Jpi^T, with Jpi the numerical Jacobian of the
    # perspective map at the mean and Sigma built from scipy's quaternion rotation.
    rng = np.random.default_rng(7)
    cam = scenes.orbit_camera(0.7, 0.3, 4.0, 320, 240)
    Rc = cam.R.astype(np.float64)
    tc = cam.t.astype(np.float64)
    for trial in range(20):
        p = rng.uniform(-0.5, 0.5, 3).astype(np.float32)
        s = np.exp(rng.normal(-3, 0.5, 3)).astype(np.float32)
        q = rng.standard_normal(4).astype(np.float32)  # unnormalised on purpose
        sc = _one(p, s, q, [0.7])
        pr = oracle.project(sc, cam, P)[0]
        if pr[F["vis"]] == 0:
            continue
        qd = q.astype(np.float64)
        Rq = Rotation.from_quat([qd[1], qd[2], qd[3], qd[0]]).as_matrix()
        Sig = Rq @ np.diag(s.astype(np.float64) ** 2) @ Rq.T

        def proj(x):
            pc = Rc @ x + tc
            return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

        pd = p.astype(np.float64)
        Jp = np.zeros((2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jp[:, k] = (proj(pd + e) - proj(pd - e)) / (2 * h)
        ref = Jp @ Sig @ Jp.T
        got = np.array([[pr[F["sxx"]], pr[F["sxy"]]], [pr[F["sxy"]], pr[F["syy"]]]]) - np.float64(np.float32(0.3)) * np.eye(2)
        assert np.abs(got - ref).max() < 1e-6 * np.abs(ref).max()
        assert np.allclose(proj(pd), [pr[F["u"]], pr[F["v"]]], atol=1e-9)


def test_culling_rules():
    cam = scenes.plain_view()
    s = [0.05, 0.05, 0.05]
    # behind the near plane (camera z = 0.1 < 0.2)
    assert oracle.project(_one([0, 0, -3.9], s, [1, 0, 0, 0], [0.9]), cam, P)[0][F["vis"]] == 0
    # opacity below 1/255
    assert oracle.project(_one([0, 0, 0], s, [1, 0, 0, 0], [0.003]), cam, P)[0][F["vis"]] == 0
    # outside the 1.3x guard window
    assert oracle.project(_one([4.0, 0, 0], s, [1, 0, 0, 0], [0.9]), cam, P)[0][F["vis"]] == 0
    # zero quaternion
    assert oracle.project(_one([0, 0, 0], s, [0, 0, 0, 0], [0.9]), cam, P)[0][F["vis"]] == 0
    # non-finite parameter
    assert oracle.project(_one([np.nan, 0, 0], s, [1, 0, 0, 0], [0.9]), cam, P)[0][F["vis"]] == 0
    # low opacity shrinks the support: q_max = 2 ln(o / alpha_min)
    pr = oracle.project(_one([0, 0, 0], s, [1, 0, 0, 0], [0.1]), cam, P)[0]
    a_min = np.float64(np.float32(1 / 255))
    assert abs(pr[F["qmax"]] - 2 * np.log(np.float64(np.float32(0.1)) / a_min)) < 1e-12


# ----------------------------------------------------------------------------------------------
# Compositing (eq. render-gs)
# ----------------------------------------------------------------------------------------------

Y00 = 0.5 / np.sqrt(np.pi)


def _dc_colour(sc):
    """Colour of a degree-0 scene from the closed form of Y_00 (a constant 1 / (2 sqrt(pi)))."""
    return np.maximum(sc.sh.astype(np.float64).reshape(3, -1) * Y00 + 0.5, 0.0)


# With the plain 128x96 view (R = I, t = (0, 0, 4), f = 100, c = (64, 48)), a mean at world
# (-2^-6, -2^-6, -0.875) has camera depth 3.125 and projects exactly onto the centre of pixel
# (63, 47): 100 * (-0.015625) / 3.125 = -0.5. The same holds at world (-2^-5, -2^-5, 2.25)
# (depth 6.25). There q = 0 and alpha equals the opacity exactly.
NEAR = [-0.015625, -0.015625, -0.875]
FAR = [-0.03125, -0.03125, 2.25]


def test_two_gaussian_closed_form():
    cam = scenes.plain_view()
    sc = _one([FAR, NEAR], [[0.05] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.75, 0.625], [[0.9, 0.2, 0.1], [0.1, 0.8, 0.3]])
    pr = oracle.project(sc, cam, P)
    assert pr[0, F["u"]] == 63.5 and pr[1, F["u"]] == 63.5 and pr[1, F["v"]] == 47.5
    out = oracle.render(sc, cam, P, pixels=(np.array([63]), np.array([47])))
    c = _dc_colour(sc)
    ref = 0.625 * c[:, 1] + (1 - 0.625) * 0.75 * c[:, 0]
    assert np.abs(out["rgb"][0] - ref).max() < 1e-15
    assert out["T"][0] == (1 - 0.75) * (1 - 0.625)
    assert out["ncomp"][0] == 2


def test_stop_rule_closed_form():
    # 20 identical Gaussians with alpha = 0.5 exactly at pixel (63, 47): T after k of them is
    # 2^-k. The 14th takes T below t_min = 1e-4 (2^-13 = 1.2e-4, 2^-14 = 6.1e-5); it is
    # composited and the ray ends there: 14 entries, T_final = 2^-14.
    cam = scenes.plain_view()
    n = 20
    sc = _one([NEAR] * n, [[0.02] * 3] * n, [[1, 0, 0, 0]] * n, [0.5] * n, [[1, 1, 1]] * n)
    out = oracle.render(sc, cam, P, pixels=(np.array([63]), np.array([47])))
    assert out["ncomp"][0] == 14
    assert out["T"][0] == 2.0 ** -14
    c = _dc_colour(sc)[0, 0]
    assert abs(out["rgb"][0][0] - c * (1 - 2.0 ** -14)) < 1e-15


def test_white_scene_identities():
    # colour 1 everywhere: with bg = 1 the image is exactly 1 (weights telescope to 1 - T);
    # with bg = 0 it equals 1 - T_final per pixel.
    sc = scenes.uniform_cube_scene(300, seed=11)
    sc.sh[:] = np.float32(0.5 * 2 * np.sqrt(np.pi))
    cam = scenes.plain_view()
    pr = oracle.project(sc, cam, P)
    c = pr[pr[:, F["vis"]] == 1, F["r"]]
    eps = np.abs(c - 1).max()
    assert eps < 1e-7
    w = oracle.render(sc, cam, P)
    assert np.abs(w["rgb"] - (1 - w["T"])[None]).max() < 2 * eps + 1e-14
    Pw = scenes.Params(bg=[1.0, 1.0, 1.0])
    w1 = oracle.render(sc, cam, Pw)
    assert np.abs(w1["rgb"] - 1).max() < 2 * eps + 1e-14
    assert (w["T"] < 0.5).sum() > 100  # the scene is not trivially transparent


def test_permutation_invariance():
    sc = scenes.uniform_cube_scene(500, seed=3)
    cam = scenes.plain_view()
    pr = oracle.project(sc, cam, P)
    d = pr[pr[:, F["vis"]] == 1, F["depth32"]]
    assert len(np.unique(d)) == len(d)  # distinct FP32 depths: the order is unique
    perm = np.random.default_rng(0).permutation(sc.n)
    a = oracle.render(sc, cam, P)
    b = oracle.render(sc.subset(perm), cam, P)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["T"], b["T"])


def test_alpha_clamp():
    # opacity 1 at q = 0: o * G = 1 is clamped to alpha_max = 0.99
    cam = scenes.plain_view()
    sc = _one([NEAR], [[0.05] * 3], [[1, 0, 0, 0]], [1.0], [[1, 1, 1]])
    out = oracle.render(sc, cam, P, pixels=(np.array([63]), np.array([47])))
    assert out["T"][0] == 1 - np.float64(np.float32(0.99))


def test_depth_tie_breaks_by_index():
    # two Gaussians at the same depth and place, different colours: the lower index is in front
    cam = scenes.plain_view()
    sc = _one([NEAR, NEAR], [[0.05] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.5, 0.5], [[1, 0, 0], [0, 0, 1]])
    c = _dc_colour(sc)
    out = oracle.render(sc, cam, P, pixels=(np.array([63]), np.array([47])))
    assert np.abs(out["rgb"][0] - (0.5 * c[:, 0] + 0.25 * c[:, 1])).max() < 1e-15
    out2 = oracle.render(sc.subset([1, 0]), cam, P, pixels=(np.array([63]), np.array([47])))
    assert np.abs(out2["rgb"][0] - (0.5 * c[:, 1] + 0.25 * c[:, 0])).max() < 1e-15


# ----------------------------------------------------------------------------------------------
# Tiles: the rectangle is conservative, so every pixel's support lies in its tile's list.
# ----------------------------------------------------------------------------------------------

@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_tile_lists_cover_every_support(tile):
    sc = scenes.uniform_cube_scene(400, seed=4)
    cam = scenes.Camera(np.eye(3, dtype=np.float32), np.float32([0, 0, 4]), 100.0, 100.0, 61.0, 45.0, 122, 90)
    pr = oracle.project(sc, cam, P, tile=tile)
    keys, vals = oracle.pairs([pr[:, F["depth32"]]], [oracle.rects_of(pr)], [(cam.width, cam.height)], tile)
    tiles_x = -(-cam.width // tile[0])
    lists = {}
    for k, v in zip(keys, vals):
        lists.setdefault(int(k >> np.uint64(32)), []).append(int(v))
    vis = np.nonzero(pr[:, F["vis"]] == 1)[0]
    for py in range(0, cam.height, 3):
        for px in range(0, cam.width, 3):
            dx, dy = px + 0.5 - pr[vis, F["u"]], py + 0.5 - pr[vis, F["v"]]
            q = pr[vis, F["ca"]] * dx * dx + 2 * pr[vis, F["cb"]] * dx * dy + pr[vis, F["cc"]] * dy * dy
            sup = set(vis[q <= pr[vis, F["qmax"]]].tolist())
            t = (py // tile[1]) * tiles_x + px // tile[0]
            assert sup <= set(lists.get(t, [])), (px, py)
    # the lists are sorted by (tile, depth, index)
    d = np.asarray(keys & np.uint64(0xFFFFFFFF), np.uint32).view(np.float32)
    t = keys >> np.uint64(32)
    for a in range(len(keys) - 1):
        assert (t[a], d[a], vals[a]) < (t[a + 1], d[a + 1], vals[a + 1])


# ----------------------------------------------------------------------------------------------
# Tile rectangle (Sec. 3.2 bins each projected Gaussian into screen tiles; the rule is a reading:
# the support's exact bounding box, hx = sqrt(q_max Sigma'_xx), hy = sqrt(q_max Sigma'_yy),
# widened by 2^-16 px, floored to tiles and clamped to the grid). Each case below computes the
# half-extents and the rectangle in closed form from the scene's numbers, not from the oracle.
# ----------------------------------------------------------------------------------------------

EPS_RECT = 2.0 ** -16
LOWPASS = np.float64(np.float32(0.3))
A_MIN = np.float64(np.float32(1 / 255))


def _axis_aligned_extent(world, s, opac, cam):
    """Closed form for R = I, t = (0, 0, 4) and an identity rotation: Sigma = diag(s^2),
    J = [[f/z, 0, -f x/z^2], [0, f/z, -f y/z^2]] at camera-space (x, y, z) = world + t."""
    x, y, z = (np.float64(np.float32(world[0])), np.float64(np.float32(world[1])),
               np.float64(np.float32(world[2])) + 4.0)
    a, b, c = np.float64(np.float32(s[0])) ** 2, np.float64(np.float32(s[1])) ** 2, np.float64(np.float32(s[2])) ** 2
    f = 100.0
    sxx = (f / z) ** 2 * a + (f * x / z ** 2) ** 2 * c + LOWPASS
    syy = (f / z) ** 2 * b + (f * y / z ** 2) ** 2 * c + LOWPASS
    qmax = min(9.0, 2.0 * np.log(np.float64(np.float32(opac)) / A_MIN))
    u, v = f * x / z + cam.cx, f * y / z + cam.cy
    return u, v, np.sqrt(qmax * sxx), np.sqrt(qmax * syy), qmax


def _rect(u, v, hx, hy, cam, tile):
    tw, th = tile
    nx, ny = -(-cam.width // tw), -(-cam.height // th)
    tx0 = max(0, int(np.floor((u - hx - EPS_RECT) / tw)))
    tx1 = min(nx - 1, int(np.floor((u + hx + EPS_RECT) / tw)))
    ty0 = max(0, int(np.floor((v - hy - EPS_RECT) / th)))
    ty1 = min(ny - 1, int(np.floor((v + hy + EPS_RECT) / th)))
    count = (tx1 - tx0 + 1) * (ty1 - ty0 + 1) if (tx1 >= tx0 and ty1 >= ty0) else 0
    return (tx0, ty0, tx1, ty1), count


def _check_rect(pr, u, v, hx, hy, qmax, cam, tile):
    assert pr[F["vis"]] == 1
    assert abs(pr[F["u"]] - u) < 1e-12 * max(1.0, abs(u)) and abs(pr[F["v"]] - v) < 1e-12 * max(1.0, abs(v))
    assert abs(pr[F["qmax"]] - qmax) < 1e-12 * qmax
    assert abs(pr[F["hx"]] - hx) < 1e-12 * hx and abs(pr[F["hy"]] - hy) < 1e-12 * hy
    rect, count = _rect(u, v, hx, hy, cam, tile)
    if count:
        got = tuple(int(pr[F[k]]) for k in ("tx0", "ty0", "tx1", "ty1"))
        assert got == rect, (got, rect)
    assert int(pr[F["count"]]) == count
    return rect, count


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_tile_rect_axis_aligned_closed_form(tile):
    # q_max = kappa^2 = 9 (opacity 0.8); Sigma'_xy != 0 off the axes does not enter hx, hy
    cam = scenes.plain_view()
    counts = []
    for world, s in [((0.3, -0.2, 0.5), (0.28, 0.15, 0.1)), ((-0.45, 0.3, -1.0), (0.02, 0.31, 0.04)),
                     ((0.0, 0.0, 0.0), (0.05, 0.02, 0.07))]:
        u, v, hx, hy, qm = _axis_aligned_extent(world, s, 0.8, cam)
        assert qm == 9.0
        pr = oracle.project(_one([world], [s], [1, 0, 0, 0], [0.8]), cam, P, tile=tile)[0]
        counts.append(_check_rect(pr, u, v, hx, hy, qm, cam, tile)[1])
    assert max(counts) > 2


def test_tile_rect_low_opacity_radius():
    # opacity 0.02: q_max = 2 ln(o / alpha_min) = 2 ln(5.1) ~ 3.26 < 9 shrinks the box
    cam = scenes.plain_view()
    world, s = (0.1, 0.05, 0.2), (0.09, 0.06, 0.05)
    u, v, hx, hy, qm = _axis_aligned_extent(world, s, 0.02, cam)
    assert 3.2 < qm < 3.3
    pr = oracle.project(_one([world], [s], [1, 0, 0, 0], [0.02]), cam, P)[0]
    _check_rect(pr, u, v, hx, hy, qm, cam, (16, 16))
    # the same Gaussian at full opacity covers a wider box
    pr9 = oracle.project(_one([world], [s], [1, 0, 0, 0], [0.8]), cam, P)[0]
    assert abs(pr9[F["hx"]] / pr[F["hx"]] - np.sqrt(9.0 / qm)) < 1e-12


def test_tile_rect_clamped_to_the_grid():
    # 128 x 96 view, 16 x 16 tiles: 8 x 6 tiles. Means near (and past) the image border but
    # inside the 1.3x guard window keep their projection; the box is clamped to the grid.
    cam = scenes.plain_view()
    tile = (16, 16)
    z = 4.0
    cases = {
        "left_top": ((2.0 - 64.0) * z / 100.0, (3.0 - 48.0) * z / 100.0),        # u = 2, v = 3
        "right_bottom": ((125.0 - 64.0) * z / 100.0, (94.0 - 48.0) * z / 100.0),  # u = 125, v = 94
        "past_left": ((-12.0 - 64.0) * z / 100.0, 0.0),                           # u = -12, outside the image
    }
    got = {}
    for name, (wx, wy) in cases.items():
        world, s = (wx, wy, 0.0), (0.3, 0.3, 0.05)
        u, v, hx, hy, qm = _axis_aligned_extent(world, s, 0.8, cam)
        pr = oracle.project(_one([world], [s], [1, 0, 0, 0], [0.8]), cam, P, tile=tile)[0]
        got[name] = _check_rect(pr, u, v, hx, hy, qm, cam, tile)
    assert got["left_top"][0][:2] == (0, 0) and got["right_bottom"][0][2:] == (7, 5)
    # u - hx < 0 < u + hx for the first, u + hx > 128 for the second: the clamp did act
    assert got["past_left"][0][0] == 0 and got["past_left"][1] > 0
    # a box entirely left of the image: visible per the culls, but no tile
    world, s = ((-18.0 - 64.0) * z / 100.0, 0.0, 0.0), (0.02, 0.02, 0.02)
    u, v, hx, hy, qm = _axis_aligned_extent(world, s, 0.8, cam)
    assert u + hx < 0
    pr = oracle.project(_one([world], [s], [1, 0, 0, 0], [0.8]), cam, P, tile=tile)[0]
    assert pr[F["vis"]] == 1 and pr[F["count"]] == 0


def _scale_for_right_edge(target, world, cam):
    """FP32 x-scale for which u + hx lies just below `target`, by bisection on the closed form."""
    lo, hi = np.float32(1e-3), np.float32(0.5)
    for _ in range(200):
        mid = np.float32((np.float64(lo) + np.float64(hi)) / 2)
        if mid in (lo, hi):
            break
        u, _, hx, _, _ = _axis_aligned_extent(world, (mid, 0.03, 0.03), 0.8, cam)
        if u + hx < target:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("gap", [2.0 ** -18, 2.0 ** -14])
def test_tile_rect_widening_at_a_tile_boundary(gap):
    # The right edge of the support's box placed just below the boundary x = 64 of tiles 3 and 4
    # (16-px tiles): within the 2^-16 widening (gap 2^-18) the box reaches tile 4; beyond it
    # (gap 2^-14) it stops at tile 3.
    cam = scenes.plain_view()
    world = (-0.4, 0.0, 0.0)  # u = 64 - 10 = 54
    target = 64.0 - gap
    sx = _scale_for_right_edge(target, world, cam)
    u, v, hx, hy, qm = _axis_aligned_extent(world, (sx, 0.03, 0.03), 0.8, cam)
    edge = u + hx
    # FP32 steps of the scale move the edge by ~1e-6 px: the bisection lands within 2^-19 of it
    assert target - 2.0 ** -19 < edge < target + 1e-9 and edge < 64.0
    pr = oracle.project(_one([world], [(sx, 0.03, 0.03)], [1, 0, 0, 0], [0.8]), cam, P)[0]
    rect, _ = _check_rect(pr, u, v, hx, hy, qm, cam, (16, 16))
    assert rect[2] == (4 if gap < EPS_RECT else 3)


def test_tile_rect_rotated_with_scipy():
    # Sigma = Rq diag(s^2) Rq^T with Rq from scipy's quaternion rotation, Sigma' from the
    # numerical Jacobian of the perspective map of a rotated camera; hx, hy and the rectangle
    # follow from Sigma'_xx, Sigma'_yy and q_max alone.
    rng = np.random.default_rng(17)
    cam = scenes.orbit_camera(0.9, 0.35, 4.0, 320, 240)
    Rc, tc = cam.R.astype(np.float64), cam.t.astype(np.float64)

    def proj(x):
        pc = Rc @ x + tc
        return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

    checked = 0
    for trial in range(60):
        p = rng.uniform(-0.8, 0.8, 3).astype(np.float32)
        s = np.exp(rng.normal(-2.5, 0.6, 3)).astype(np.float32)
        q = rng.standard_normal(4).astype(np.float32)
        o = np.float32(rng.choice([0.8, 0.03]))
        for tile in [(16, 16), (8, 32)]:
            pr = oracle.project(_one(p, s, q, [o]), cam, P, tile=tile)[0]
            if pr[F["vis"]] == 0:
                continue
            qd = q.astype(np.float64)
            Rq = Rotation.from_quat([qd[1], qd[2], qd[3], qd[0]]).as_matrix()
            Sig = Rq @ np.diag(s.astype(np.float64) ** 2) @ Rq.T
            pd = p.astype(np.float64)
            Jp = np.zeros((2, 3))
            for k in range(3):
                e = np.zeros(3)
                e[k] = 1e-6
                Jp[:, k] = (proj(pd + e) - proj(pd - e)) / 2e-6
            Sp = Jp @ Sig @ Jp.T + LOWPASS * np.eye(2)
            qm = min(9.0, 2.0 * np.log(np.float64(o) / A_MIN))
            hx, hy = np.sqrt(qm * Sp[0, 0]), np.sqrt(qm * Sp[1, 1])
            u, v = proj(pd)
            assert abs(pr[F["hx"]] - hx) < 1e-7 * hx and abs(pr[F["hy"]] - hy) < 1e-7 * hy
            # rectangle from the reference box, unless an edge lies within 1e-5 px of a tile line
            edges = np.array([(u - hx - EPS_RECT) / tile[0], (u + hx + EPS_RECT) / tile[0],
                              (v - hy - EPS_RECT) / tile[1], (v + hy + EPS_RECT) / tile[1]])
            if np.any(np.abs(edges - np.round(edges)) * min(tile) < 1e-5):
                continue
            rect, count = _rect(u, v, hx, hy, cam, tile)
            assert int(pr[F["count"]]) == count
            if count:
                assert tuple(int(pr[F[k]]) for k in ("tx0", "ty0", "tx1", "ty1")) == rect
            checked += 1
    assert checked > 60


def test_half_extents_bound_the_support_ellipse():
    # hx, hy are the exact half-widths of {d : d^T conic d <= q_max}: the boundary points
    # sqrt(q_max) V diag(lambda^-1/2) (cos t, sin t) (numpy's eigen-decomposition of the
    # oracle's conic) reach +-hx in x and +-hy in y and never beyond.
    sc = scenes.mixture_scene(3000, seed=5)
    cam = scenes.orbit_camera(0.2, 0.1, 4.0, 320, 240)
    pr = oracle.project(sc, cam, P)
    vis = np.nonzero(pr[:, F["vis"]] == 1)[0]
    assert len(vis) > 200
    t = np.linspace(0, 2 * np.pi, 20001)
    circle = np.stack([np.cos(t), np.sin(t)])
    for i in vis[:200]:
        C = np.array([[pr[i, F["ca"]], pr[i, F["cb"]]], [pr[i, F["cb"]], pr[i, F["cc"]]]])
        lam, V = np.linalg.eigh(C)
        d = np.sqrt(pr[i, F["qmax"]]) * (V @ (circle / np.sqrt(lam)[:, None]))
        ex, ey = np.abs(d[0]).max(), np.abs(d[1]).max()
        # dense sampling reaches the extreme to second order in the angle step
        assert ex <= pr[i, F["hx"]] * (1 + 1e-9) and ex >= pr[i, F["hx"]] * (1 - 1e-7)
        assert ey <= pr[i, F["hy"]] * (1 + 1e-9) and ey >= pr[i, F["hy"]] * (1 - 1e-7)


def test_pairs_brute_force_per_tile():
    sc = scenes.uniform_cube_scene(150, seed=9)
    cams = [scenes.plain_view(), scenes.orbit_camera(0.4, 0.2, 4.0, 70, 50, fx=60.0)]
    tile = (16, 16)
    prs = [oracle.project(sc, c, P, tile) for c in cams]
    keys, vals = oracle.pairs([p[:, F["depth32"]] for p in prs], [oracle.rects_of(p) for p in prs],
                              [(c.width, c.height) for c in cams], tile)
    ref = []
    off = 0
    for c, p in zip(cams, prs):
        tx_n, ty_n = -(-c.width // 16), -(-c.height // 16)
        for ty in range(ty_n):
            for tx in range(tx_n):
                inside = [i for i in range(sc.n) if p[i, F["vis"]] == 1 and p[i, F["count"]] > 0
                          and p[i, F["tx0"]] <= tx <= p[i, F["tx1"]] and p[i, F["ty0"]] <= ty <= p[i, F["ty1"]]]
                inside.sort(key=lambda i: (np.float32(p[i, F["depth32"]]), i))
                ref += [(off + ty * tx_n + tx, i) for i in inside]
        off += tx_n * ty_n
    assert [(int(k >> np.uint64(32)), int(v)) for k, v in zip(keys, vals)] == ref


# ----------------------------------------------------------------------------------------------
# Importance (eq. importance-score) and cluster lists (eq. importance-score-vis)
# ----------------------------------------------------------------------------------------------

def test_importance_properties():
    sc = scenes.uniform_cube_scene(2000, seed=12)
    sc.scale[:] *= 2  # dense enough that some Gaussians are hidden from every view
    cams = [scenes.orbit_camera(a, 0.1, 4.0, 64, 48, fx=50.0) for a in (0.0, 1.0, 2.5)]
    h = oracle.importance(sc, cams, P)
    # max is independent of how often a view occurs
    h2 = oracle.importance(sc, cams + cams[:2], P)
    assert np.array_equal(h, h2)
    # monotone in the view set
    assert np.all(oracle.importance(sc, cams[:2], P) <= h)
    # removing exactly the never-composited Gaussians leaves every training render bit-identical
    keep = np.nonzero(h > 0)[0]
    assert 0 < len(keep) < sc.n
    for c in cams:
        a = oracle.render(sc, c, P)
        b = oracle.render(sc.subset(keep), c, P)
        assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["T"], b["T"])
    # the mask follows Sec. 3.3 literally: h < t is pruned, equality is kept
    m = oracle.prune_mask(np.array([0.0, 0.01, 0.0099, 0.02]), 0.01)
    assert m.tolist() == [True, False, True, False]


def test_cluster_bits_partition_identity():
    sc = scenes.uniform_cube_scene(300, seed=13)
    cams = [scenes.orbit_camera(a, e, 4.0, 48, 40, fx=40.0) for a, e in [(0, 0), (0.3, 0.1), (2, 0.2), (2.2, 0), (4, 0.1)]]
    assign = [0, 0, 1, 1, 2]
    t = 0.01
    bits = oracle.cluster_bits(sc, cams, assign, 3, P, t)
    h = oracle.importance(sc, cams, P)
    assert np.array_equal(bits.any(0), h > t)
    one = oracle.cluster_bits(sc, cams, [0] * 5, 1, P, t)
    assert np.array_equal(one[0], h > t)
    # a view rendered from its cluster's list at t -> 0+ is identical to the unfiltered render
    bits0 = oracle.cluster_bits(sc, cams, assign, 3, P, 0.0)
    for v, c in enumerate(cams):
        a = oracle.render(sc, c, P)
        b = oracle.render(sc.subset(np.nonzero(bits0[assign[v]])[0]), c, P)
        assert np.array_equal(a["rgb"], b["rgb"])


# ----------------------------------------------------------------------------------------------
# Gradients: analytic oracle backward vs central finite differences of the oracle forward.
# ----------------------------------------------------------------------------------------------

def _loss_and_fp(sc, cam, w):
    out = oracle.render(sc, cam, P, fingerprint=True)
    return float((out["rgb"] * w).sum()), out["fp"]


@pytest.mark.parametrize("deg", [0, 3])
def test_gradient_vs_central_differences(deg):
    rng = np.random.default_rng(21 + deg)
    n = 12
    base = scenes.uniform_cube_scene(n, seed=30 + deg)
    mean = (base.mean * 0.6).astype(np.float32)
    scale = np.exp(rng.normal(-2.2, 0.4, (3, n))).astype(np.float32)
    quat = rng.standard_normal((4, n)).astype(np.float32)
    opac = rng.uniform(0.3, 0.9, n).astype(np.float32)
    sh = rng.normal(0, 0.3, ((deg + 1) ** 2 * 3, n)).astype(np.float32)
    sh[0:3] += 0.6
    cam = scenes.orbit_camera(0.3, 0.2, 4.0, 40, 32, fx=45.0)
    sc = scenes.Scene(mean, scale, quat, opac, sh, deg)
    w = rng.uniform(-1, 1, (3, cam.height, cam.width))
    g = oracle.render_bwd(sc, cam, P, w)
    checked = 0
    for name, arr in [("mean", "mean"), ("scale", "scale"), ("quat", "quat"), ("opacity", "opacity"), ("sh", "sh")]:
        A = getattr(sc, arr)
        flat = A.reshape(-1)
        for j in rng.choice(flat.size, min(flat.size, 24), replace=False):
            x0 = float(flat[j])
            h = 1e-6 * max(abs(x0), 1e-2)
            vals, fps = [], []
            for sgn in (+1, -1):
                B = A.astype(np.float64).copy().reshape(-1)
                B[j] = x0 + sgn * h
                sc2 = scenes.Scene(**{**sc.__dict__, arr: B.reshape(A.shape)})
                # keep FP64 inputs: the oracle widens whatever it gets
                L, fp = _loss_and_fp(sc2, cam, w)
                vals.append(L)
                fps.append(fp)
            if not np.array_equal(fps[0], fps[1]):
                continue  # a discrete decision changed inside the stencil
            fd = (vals[0] - vals[1]) / (2 * h)
            an = g[name].reshape(-1)[j]
            scale_ref = np.abs(g[name]).max() + 1e-12
            assert abs(fd - an) <= 1e-5 * scale_ref + 1e-6 * abs(an), (name, j, fd, an)
            checked += 1
    assert checked > 60
