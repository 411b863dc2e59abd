"""Pins for the FP64 brute-force oracle (k-NN definition, Hercules Sec. 2).

The oracle is checked against things other than itself: scipy's exact
KD-tree search (a library routine for the same definition), hand-built
collections whose answer is known in closed form, planted exact ties (which
must be broken by the smaller id), and its own numpy twin.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import brute
from paper_2212_13297_amd import datagen as G


@pytest.mark.parametrize("N,n,k", [(50, 8, 1), (300, 16, 7), (1000, 64, 10), (257, 256, 25)])
def test_matches_kdtree(N, n, k):
    rng = np.random.default_rng(N + n)
    x = rng.standard_normal((N, n)).astype(np.float32)
    q = rng.standard_normal((5, n)).astype(np.float32)
    ids, d2 = brute.knn(x, q, k)
    dist, idx = cKDTree(x.astype(np.float64)).query(q.astype(np.float64), k=k)
    dist = np.asarray(dist).reshape(5, k)
    idx = np.asarray(idx).reshape(5, k)
    # continuous random data: no ties, so the orders agree exactly
    np.testing.assert_array_equal(ids, idx)
    np.testing.assert_allclose(d2, dist ** 2, rtol=1e-12)


def test_numpy_twin_and_thread_count():
    x = G.random_walks(3000, 128)
    q, _, _ = G.workload(x, [1, 10], 4)
    a = brute.knn(x, q, 9, threads=1)
    b = brute.knn(x, q, 9, threads=7)
    c = brute.knn_numpy(x, q, 9)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[0], c[0])
    np.testing.assert_allclose(a[1], c[1], rtol=1e-12)


def test_closed_form_axis_points():
    # x_i = i * e_0 (i = 0..N-1); the query t * e_0 has d(i) = (i - t)^2.
    N, n = 40, 16
    x = np.zeros((N, n), np.float32)
    x[:, 0] = np.arange(N)
    q = np.zeros((1, n), np.float32)
    q[0, 0] = 10.25
    ids, d2 = brute.knn(x, q, 5)
    np.testing.assert_array_equal(ids[0], [10, 11, 9, 12, 8])
    np.testing.assert_array_equal(d2[0], [0.0625, 0.5625, 1.5625, 3.0625, 5.0625])


def test_ties_broken_by_id():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((100, 32)).astype(np.float32)
    x[70] = x[3]          # exact duplicates of row 3
    x[41] = x[3]
    q = x[3:4].copy()
    ids, d2 = brute.knn(x, q, 3)
    np.testing.assert_array_equal(ids[0], [3, 41, 70])
    np.testing.assert_array_equal(d2[0], [0.0, 0.0, 0.0])
    # a query equidistant from two rows (mirror images around it)
    x2 = np.zeros((6, 4), np.float32)
    x2[5, 0] = 1.0
    x2[2, 0] = -1.0
    x2[0] = 5.0
    x2[1] = 6.0
    x2[3] = 7.0
    x2[4] = 8.0
    ids, d2 = brute.knn(x2, np.zeros((1, 4), np.float32), 2)
    np.testing.assert_array_equal(ids[0], [2, 5])
    np.testing.assert_array_equal(d2[0], [1.0, 1.0])


def test_k_equals_n_is_full_sort():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((33, 8)).astype(np.float32)
    q = rng.standard_normal((2, 8)).astype(np.float32)
    ids, d2 = brute.knn(x, q, 33)
    for i in range(2):
        full = ((x.astype(np.float64) - q[i].astype(np.float64)) ** 2).sum(1)
        assert sorted(ids[i].tolist()) == list(range(33))
        assert np.all(np.diff(d2[i]) >= 0)
        np.testing.assert_allclose(d2[i], full[ids[i]], rtol=1e-12)


def test_pair_dist_matches_knn():
    x = G.random_walks(500, 64)
    q, _, _ = G.workload(x, [5], 3)
    ids, d2 = brute.knn(x, q, 4)
    qi = np.repeat(np.arange(3), 4)
    got = brute.pair_dist(x, q, qi, ids.reshape(-1))
    np.testing.assert_array_equal(got, d2.reshape(-1))


def test_invalid_arguments():
    x = np.zeros((5, 4), np.float32)
    q = np.zeros((1, 4), np.float32)
    with pytest.raises(ValueError):
        brute.knn(x, q, 6)
    with pytest.raises(ValueError):
        brute.knn(x, q, 0)
    with pytest.raises(ValueError):
        brute.knn(x, np.zeros((1, 5), np.float32), 1)


def test_knn_chunked_equals_whole_collection():
    # Ties across chunk boundaries (exact copies in different chunks) must be
    # broken by the global id, and a chunk smaller than k must not truncate.
    rng = np.random.default_rng(7)
    x = rng.standard_normal((700, 24)).astype(np.float32)
    x[650] = x[3]
    x[420] = x[3]
    q = rng.standard_normal((6, 24)).astype(np.float32)
    q[0] = x[3]
    for k in (1, 5, 9):
        whole = brute.knn(x, q, k)
        parts = brute.knn_chunked([x[:4], x[4:421], x[421:422], x[422:]], q, k)
        assert np.array_equal(whole[0], parts[0]) and np.array_equal(whole[1], parts[1])
        twin = brute.knn_numpy(x, q, k)
        assert np.array_equal(parts[0], twin[0])
    assert list(brute.knn_chunked([x[:100], x[100:]], q[:1], 3)[0][0]) == [3, 420, 650]
