"""Pins of the FP64 initialisation oracle (Sec. 3.2): nearest-neighbour distances against
scipy's k-d tree, closed forms on lattices and small configurations, coincident points, and
the SH DC coefficient against scipy's spherical harmonic Y_0^0."""
import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial import cKDTree

from oracle import init as OI


def test_nn_matches_kdtree():
    rng = np.random.default_rng(0)
    p = rng.uniform(-3, 3, (3, 1500)).astype(np.float32)
    d, _ = cKDTree(p.T.astype(np.float64)).query(p.T.astype(np.float64), k=2)
    np.testing.assert_allclose(OI.nn_distance(p), d[:, 1].astype(np.float32), rtol=1e-6)


def test_lattice_spacing():
    """Every point of a cubic lattice of spacing a has nearest distance a."""
    a = 0.375
    g = np.arange(5, dtype=np.float64) * a
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    p = np.stack([x.ravel(), y.ravel(), z.ravel()]).astype(np.float32)
    assert np.all(OI.nn_distance(p) == np.float32(a))


def test_small_configurations():
    two = np.array([[0, 3], [0, 4], [0, 0]], np.float32)
    assert np.all(OI.nn_distance(two) == 5.0)
    assert np.isinf(OI.nn_distance(np.zeros((3, 1), np.float32))[0])
    assert np.all(np.isinf(OI.nn_distance(np.ones((3, 4), np.float32))))  # all coincident
    # coincident copies are not neighbours: the nearest point at another position counts
    p = np.array([[0, 0, 2], [0, 0, 0], [0, 0, 0]], np.float32)
    assert list(OI.nn_distance(p)) == [2.0, 2.0, 2.0]


def test_invariances():
    rng = np.random.default_rng(1)
    p = rng.uniform(-1, 1, (3, 400)).astype(np.float32)
    s = OI.nn_distance(p)
    perm = rng.permutation(400)
    assert np.array_equal(OI.nn_distance(p[:, perm]), s[perm])
    q = (p.astype(np.float64) * 2.0).astype(np.float32)  # exact scaling by 2
    assert np.array_equal(OI.nn_distance(q), 2 * s)


def test_init_constants_and_dc_colour():
    rng = np.random.default_rng(2)
    p = rng.uniform(-1, 1, (3, 50)).astype(np.float32)
    c = rng.uniform(0, 1, (3, 50)).astype(np.float32)
    mean, scale, quat, opac, sh = OI.init_gaussians(p, c, 3)
    assert np.array_equal(mean, p) and sh.shape == (48, 50)
    assert np.all(scale[0] == scale[1]) and np.all(scale[1] == scale[2])
    assert np.all(quat[0] == 1) and np.all(quat[1:] == 0) and np.all(opac == np.float32(0.1))
    assert np.all(sh[3:] == 0)
    y00 = float(np.real(sps.sph_harm_y(0, 0, 0.3, 0.7)))
    assert OI.Y00 == pytest.approx(y00, rel=1e-15)
    # colour model c = max(0, k Y00 + 1/2) returns the given colour
    np.testing.assert_allclose(sh[0:3].astype(np.float64) * y00 + 0.5, c, atol=1e-7)
