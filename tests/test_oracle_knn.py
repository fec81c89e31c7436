"""Pins of the reference neighbour selection (section 3, Fig. 2; neighbour cap, section 5).

The definition: every other agent closer than the observation radius, nearest
first (ties by id), at most K.  The reference takes the distance decision in
float32.  Pinned against scipy's KD-tree in float64: the sets must be equal
except where a distance sits within 1e-6 m of the radius or of another
selected distance (there float32 and float64 may order differently).
The paper's binned read (3x3 bins) must give exactly the definition's lists.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1908_10107_amd import scenes

BAND = 1e-6


def kdtree_lists(pos, nd, k):
    pts = pos.T.astype(np.float64)
    tree = cKDTree(pts)
    out = []
    for i, nb in enumerate(tree.query_ball_point(pts, nd * (1 + 1e-6))):
        nb = np.array([j for j in nb if j != i], np.int64)
        d = np.linalg.norm(pts[nb] - pts[i], axis=1) if nb.size else np.zeros(0)
        order = np.lexsort((nb, d))
        out.append((nb[order], d[order]))
    return out


@pytest.mark.parametrize("seed,n,side,nd,k", [(0, 600, 20.0, 3.0, 16), (1, 800, 40.0, 5.0, 10),
                                              (2, 300, 6.0, 2.0, 8), (3, 50, 100.0, 5.0, 4)])
def test_brute_matches_kdtree_outside_bands(oracle_lib, seed, n, side, nd, k):
    rng = np.random.default_rng(seed)
    pos = ((rng.random((n, 2)) - 0.5) * side).T.astype(np.float32)
    ref = kdtree_lists(pos, nd, k)
    checked = 0
    for i in range(n):
        ids, d2 = oracle_lib.knn_brute(pos, i, nd, k)
        nb, d = ref[i]
        inside = nb[d < nd]
        dd = d[d < nd]
        # ambiguous if any distance is within BAND of the radius or of the K-th
        near_cut = np.any(np.abs(d - nd) < BAND)
        near_k = len(dd) > k and abs(dd[k] - dd[k - 1]) < BAND
        if near_cut or near_k:
            continue
        checked += 1
        assert np.array_equal(ids, inside[:k]), i
        np.testing.assert_allclose(np.sqrt(d2.astype(np.float64)), dd[:k], rtol=1e-6, atol=1e-6)
    assert checked > 0.95 * n


def test_duplicate_points_tie_by_id(oracle_lib):
    pos = np.array([[0, 1, 1, 1, 1, -1], [0, 0, 0, 0, 0, 0]], np.float32)
    ids, d2 = oracle_lib.knn_brute(pos, 0, 5.0, 3)
    assert list(ids) == [1, 2, 3]
    ids, _ = oracle_lib.knn_brute(pos, 2, 5.0, 10)
    assert list(ids) == [1, 3, 4, 0, 5]


def test_strict_radius(oracle_lib):
    pos = np.array([[0, 3, -2], [0, 0, 0]], np.float32)
    ids, _ = oracle_lib.knn_brute(pos, 0, 3.0, 4)
    assert list(ids) == [2]          # exactly 3 m away is not observed


@pytest.mark.parametrize("maker", ["uniform", "dense", "ring", "clustered"])
def test_binned_equals_definition(oracle_lib, maker):
    rng = np.random.default_rng(7)
    if maker == "uniform":
        w = scenes.uniform_rsa(n=1024)
        pos, nd, k = w.pos, 5.0, 10
    elif maker == "dense":
        w = scenes.dense_uniform(n=2048)
        pos, nd, k = w.pos, 3.0, 16
    elif maker == "ring":
        w = scenes.ring(n=4096, radius_m=80.0)
        pos, nd, k = w.pos, 5.0, 10
    else:
        c = rng.normal(size=(20, 2)) * 30
        pos = (c[rng.integers(0, 20, 1500)] + rng.normal(size=(1500, 2)) * 1.5).T
        pos = pos.astype(np.float32)
        nd, k = 4.0, 12
    n = pos.shape[1]
    binned = oracle_lib.knn_binned(pos, nd, k)
    for i in range(n):
        ids, _ = oracle_lib.knn_brute(pos, i, nd, k)
        row = binned[i]
        assert np.array_equal(row[row >= 0], ids), i
