"""Pins of the roadmap reference (oracle/roadmap.py): hand-worked neighbour lists, the tie rule,
an FP64 k-d tree cross-check, and the exactly-once property of the undirected edge list."""
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import roadmap


def test_knn_hand_line():
    # points on a line at 0, 1, 3, 6, 10: neighbour lists worked out by hand
    x = np.array([[0, 0], [1, 0], [3, 0], [6, 0], [10, 0]], np.float32)
    idx, d2 = roadmap.knn(x, 2)
    # sample 2 (at 3) has samples 0 and 3 both at distance 3: the tie goes to index 0
    np.testing.assert_array_equal(idx, [[1, 2], [0, 2], [1, 0], [2, 4], [3, 2]])
    np.testing.assert_array_equal(d2, [[1, 9], [1, 4], [4, 9], [9, 16], [16, 49]])


def test_knn_ties_go_to_lower_index():
    # four corners of a unit square around the query at the centre: all at equal distance
    x = np.array([[0.5, 0.5], [1, 1], [0, 0], [1, 0], [0, 1]], np.float32)
    idx, d2 = roadmap.knn(x, 3, rows=[0])
    np.testing.assert_array_equal(idx[0], [1, 2, 3])
    assert np.all(d2[0] == np.float32(0.5))


def test_knn_matches_fp64_kdtree():
    g = np.random.default_rng(3)
    x = g.uniform(-2.9, 2.9, (700, 7)).astype(np.float32)
    k = 9
    idx, d2 = roadmap.knn(x, k)
    dist, nb = cKDTree(x.astype(np.float64)).query(x.astype(np.float64), k + 1)
    dist, nb = dist[:, 1:], nb[:, 1:]                       # drop the sample itself
    # where the FP64 order has no near-tie at the k-th neighbour the sets must agree
    d_all = np.sqrt(((x[:, None, :].astype(np.float64) - x[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d_all, np.inf)
    srt = np.sort(d_all, axis=1)
    clear = (srt[:, k] - srt[:, k - 1]) > 1e-5
    assert clear.mean() > 0.95
    for i in np.nonzero(clear)[0]:
        assert set(idx[i]) == set(nb[i])
    np.testing.assert_allclose(np.sqrt(d2.astype(np.float64)), dist, rtol=1e-5)


def test_knn_short_rows_and_non_finite():
    # k >= n: the missing neighbours are -1 / +inf; a non-finite sample is nobody's neighbour
    x = np.array([[0, 0], [1, 0], [np.nan, 0]], np.float32)
    idx, d2 = roadmap.knn(x, 3)
    np.testing.assert_array_equal(idx, [[1, -1, -1], [0, -1, -1], [-1, -1, -1]])
    assert d2[0, 0] == 1 and np.isinf(d2[0, 1:]).all() and np.isinf(d2[2]).all()
    with pytest.raises(ValueError):
        roadmap.knn(x, 0)


def test_knn_pairs_exactly_once():
    g = np.random.default_rng(4)
    x = g.uniform(-1, 1, (300, 3)).astype(np.float32)
    idx, _ = roadmap.knn(x, 6)
    pairs = roadmap.knn_pairs(idx)
    real = pairs[pairs[:, 0] >= 0]
    und = {tuple(sorted(p)) for p in real.tolist()}
    assert len(und) == len(real)                            # no edge twice
    want = {tuple(sorted((i, int(j)))) for i in range(len(x)) for j in idx[i]}
    assert und == want                                      # every kNN edge present
    assert np.all(pairs[pairs[:, 0] < 0] == -1)


def test_knn_pairs_hand():
    # mutual neighbours 0-1 appear once (from the lower index); 2's list holds 1, whose list
    # does not hold 2, so (2, 1) is kept at slot 2*1+0
    idx = np.array([[1], [0], [1]], np.int32)
    np.testing.assert_array_equal(roadmap.knn_pairs(idx), [[0, 1], [-1, -1], [2, 1]])


# --- the FP64 definition (knn_exact), the parity reference of the GPU lists -------------------

def test_exact_hand_line():
    # the same line as above, in exact arithmetic: distances are the squared gaps
    x = np.array([[0, 0], [1, 0], [3, 0], [6, 0], [10, 0]], np.float32)
    idx, d2, nxt = roadmap.knn_exact(x, 2)
    np.testing.assert_array_equal(idx, [[1, 2], [0, 2], [1, 0], [2, 4], [3, 2]])
    np.testing.assert_array_equal(d2, [[1, 9], [1, 4], [4, 9], [9, 16], [16, 49]])
    # the third-nearest of each sample, worked out by hand
    np.testing.assert_array_equal(nxt, [36, 25, 9, 25, 81])


def test_exact_ties_go_to_lower_index():
    x = np.array([[0.5, 0.5], [1, 1], [0, 0], [1, 0], [0, 1]], np.float32)
    idx, d2, nxt = roadmap.knn_exact(x, 3, rows=[0])
    np.testing.assert_array_equal(idx[0], [1, 2, 3])
    assert np.all(d2[0] == 0.5) and nxt[0] == 0.5


def test_exact_brute_force_small():
    # an independent formulation: math.dist over every pair, sorted by (distance, index)
    import math
    g = np.random.default_rng(11)
    x = g.uniform(-2.9, 2.9, (40, 5)).astype(np.float32)
    k = 6
    idx, d2, nxt = roadmap.knn_exact(x, k)
    for i in range(len(x)):
        others = sorted((math.dist(x[i].tolist(), x[j].tolist()), j) for j in range(len(x)) if j != i)
        assert idx[i].tolist() == [j for _, j in others[:k]]
        np.testing.assert_allclose(np.sqrt(d2[i]), [d for d, _ in others[:k]], rtol=1e-14)
        assert math.isclose(math.sqrt(nxt[i]), others[k][0], rel_tol=1e-14)


def test_exact_matches_fp64_kdtree_everywhere():
    g = np.random.default_rng(3)
    x = g.uniform(-2.9, 2.9, (700, 7)).astype(np.float32)
    k = 9
    idx, d2, _ = roadmap.knn_exact(x, k)
    dist, nb = cKDTree(x.astype(np.float64)).query(x.astype(np.float64), k + 1)
    np.testing.assert_allclose(np.sqrt(d2), dist[:, 1:], rtol=1e-12)
    same = (idx == nb[:, 1:]).all(axis=1)
    assert same.mean() > 0.999                  # only exact FP64 ties may order differently


def test_exact_short_rows_and_non_finite():
    x = np.array([[0, 0], [1, 0], [np.nan, 0], [0, np.inf]], np.float32)
    idx, d2, nxt = roadmap.knn_exact(x, 3)
    np.testing.assert_array_equal(idx, [[1, -1, -1], [0, -1, -1], [-1, -1, -1], [-1, -1, -1]])
    assert d2[0, 0] == 1 and np.isinf(d2[0, 1:]).all() and np.isinf(nxt).all()


def test_fp32_order_within_the_rounding_bound():
    """The fixed-order FP32 evaluation agrees with the FP64 definition wherever the exact
    distances are separated by more than the FP32 rounding bound, and its distances are within
    that bound (the GPU tests hold the kernel to the same rule)."""
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import knn_against_exact
    g = np.random.default_rng(5)
    for n, dim, k in ((300, 7, 10), (200, 14, 32), (129, 20, 9)):
        x = g.uniform(-2.9, 2.9, (n, dim)).astype(np.float32)
        fi, fd = roadmap.knn(x, k)
        rows, ties = knn_against_exact(x, fi, fd, k)
        assert rows == n
    # a near tie the FP32 evaluation cannot resolve: two samples whose exact distances differ
    # by far less than the bound; either may come first, both must be listed
    x = np.array([[0, 0], [1, 0], [0, 1 + 2.0 ** -23]], np.float32)
    fi, fd = roadmap.knn(x, 2, rows=[0])
    _, ties = knn_against_exact(x, fi, fd, 2, rows=[0])
    assert ties == 1


def test_rounding_bound_is_not_vacuous():
    # the bound holds on random data with room to spare, and is tight within a small factor:
    # the worst observed FP32 error over many sums reaches a visible share of it
    # (in one dimension the difference, its square and the rounding of the square compound to
    # almost three units in the last place, so a bound of fewer terms fails there)
    g = np.random.default_rng(7)
    for dim, n in ((1, 1500), (2, 1000), (7, 400)):
        x = g.uniform(-2.9, 2.9, (n, dim)).astype(np.float32)
        s32 = roadmap.dist2_f32(x, x).astype(np.float64)
        s64 = roadmap.dist2_exact(x, x)
        off = ~np.eye(len(x), dtype=bool) & (s64 > 0)
        rel = np.abs(s32 - s64)[off] / s64[off]
        b = roadmap.fp32_rel_bound(dim)
        assert rel.max() <= b, dim
        assert rel.max() >= 0.25 * b, dim
