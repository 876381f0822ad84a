"""Pins of the FP64 Lloyd oracle: separated groups are recovered with their exact means, a
one-dimensional two-cluster case converges to the closed-form split, an empty cluster moves to
the farthest point, and permuting the points permutes the assignment."""
import numpy as np

from oracle import kmeans as OK


def test_separated_groups_recovered():
    rng = np.random.default_rng(0)
    truth = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]], float)
    lab = np.repeat(np.arange(4), 40)
    pos = truth[lab] + rng.normal(0, 0.3, (160, 3))
    c, a, _ = OK.lloyd(pos, pos[[0, 40, 80, 120]], 50)
    for j in range(4):
        assert len(set(a[lab == j])) == 1
        np.testing.assert_allclose(c[a[lab == j][0]], pos[lab == j].mean(0), rtol=1e-14)


def test_one_dimensional_split():
    xs = np.array([0.0, 1.0, 2.0, 10.0, 11.0, 12.0])
    pos = np.stack([xs, np.zeros(6), np.zeros(6)], 1)
    c, a, _ = OK.lloyd(pos, pos[[0, 1]], 20)
    assert list(a) == [0, 0, 0, 1, 1, 1]
    np.testing.assert_allclose(c[:, 0], [1.0, 11.0])


def test_empty_cluster_moves_to_farthest_point():
    pos = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [9, 0, 0]], float)
    # centre 1 starts far away and receives no point in the first assignment
    c, a, _ = OK.lloyd(pos, np.array([[1.0, 0, 0], [100.0, 0, 0]]), 1)
    np.testing.assert_allclose(c[1], [9.0, 0, 0])
    np.testing.assert_allclose(c[0], [3.0, 0, 0])


def test_permutation_equivariance():
    rng = np.random.default_rng(1)
    pos = rng.uniform(-5, 5, (200, 3))
    init = pos[:6].copy()
    c, a, it = OK.lloyd(pos, init, 30)
    perm = rng.permutation(200)
    c2, a2, it2 = OK.lloyd(pos[perm], init, 30)
    assert np.array_equal(a2, a[perm]) and it2 == it
    np.testing.assert_allclose(c2, c, rtol=1e-12)


def test_converged_fixed_point_by_brute_force():
    """At convergence (a plain-loop check): every point's centre is its nearest one, ties to the
    lowest, and every centre is the mean of its points."""
    rng = np.random.default_rng(2)
    pos = np.concatenate([rng.normal(m, 0.5, (30, 3)) for m in ([0, 0, 0], [4, 0, 0], [0, 4, 1])])
    c, a, it = OK.lloyd(pos, pos[[0, 1, 2, 3]], 100)
    assert it < 100
    for i, p in enumerate(pos):
        best, bd = 0, None
        for j, q in enumerate(c):
            d = sum((float(p[e]) - float(q[e])) ** 2 for e in range(3))
            if bd is None or d < bd:
                best, bd = j, d
        assert a[i] == best
    for j in range(len(c)):
        mem = [pos[i] for i in range(len(pos)) if a[i] == j]
        for e in range(3):
            assert abs(sum(float(p[e]) for p in mem) / len(mem) - c[j][e]) < 1e-12


def test_max_iter_counts_updates():
    pos = np.array([[0.0, 0, 0], [1, 0, 0], [10, 0, 0], [11, 0, 0]])
    c, a, it = OK.lloyd(pos, pos[[0, 1]], 1)
    # one update from centres 0 and 1: {0} and {1, 10, 11}, then the final assignment
    assert it == 1
    np.testing.assert_allclose(c, [[0, 0, 0], [22 / 3, 0, 0]])
    assert list(a) == [0, 0, 1, 1]
    c, a, it = OK.lloyd(pos, pos[[0, 1]], 100)
    assert list(a) == [0, 0, 1, 1] and it == 2
