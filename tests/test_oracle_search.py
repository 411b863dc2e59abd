"""Pins for the oracle's serial run of the exact search (Hercules Sec. 3.4).

The paper's central claim is that the search is exact: every access path
returns the k-NN of the plain definition.  The serial FP64 filter-and-refine
must therefore equal brute force for every leaf size, seed size, threshold
setting (each path forced), k, and for planted ties.
"""
import numpy as np
import pytest

from oracle import brute, search
from paper_2212_13297_amd import datagen as G


@pytest.fixture(scope="module")
def data():
    x = G.random_walks(4000, 128, coll=3)
    q, _, _ = G.workload(x, [1, 5, 10], 2, coll=3)
    q = np.concatenate([q, G.ood_queries(2, 128, coll=3)])
    return x, q


@pytest.mark.parametrize("tau,l_max,eth,sth,k", [
    (200, 1, 0.25, 0.50, 1),
    (200, 1, 0.25, 0.50, 10),
    (50, 3, 0.0, 0.0, 5),        # always the LB_SAX path
    (1000, 0, 1.1, 0.0, 7),      # always skip-sequential after the leaf filter
    (300, 2, 0.0, 1.1, 3),       # LB_SAX computed, then skip-sequential
    (4000, 1, 0.25, 0.5, 20),    # a single leaf
    (1, 1, 0.25, 0.5, 2),        # one series per leaf
])
def test_filter_refine_equals_brute(data, tau, l_max, eth, sth, k):
    x, q = data
    idx = search.LeafIndex(x, 16, tau)
    ids, d2 = brute.knn(x, q, k)
    for i in range(len(q)):
        a, b = search.exact_knn(idx, q[i], k, l_max=l_max, eapca_th=eth, sax_th=sth)
        np.testing.assert_array_equal(a, ids[i])
        np.testing.assert_array_equal(b, d2[i])


def test_filter_refine_planted_ties():
    x = G.random_walks(1500, 64, coll=4).copy()
    x[900] = x[12]
    x[1400] = x[12]
    q = x[12:13] + np.float32(0.0)
    idx = search.LeafIndex(x, 8, 100)
    a, b = search.exact_knn(idx, q[0], 3)
    np.testing.assert_array_equal(a, [12, 900, 1400])
    np.testing.assert_array_equal(b, [0.0, 0.0, 0.0])


def test_paths_are_taken(data):
    x, q = data
    idx = search.LeafIndex(x, 16, 200)
    seen = set()
    for eth, sth in ((0.0, 0.0), (1.1, 0.0), (0.0, 1.1)):
        st = {}
        search.exact_knn(idx, q[0], 5, eapca_th=eth, sax_th=sth, stats=st)
        seen.add(st["path"])
    assert seen == {"sax", "skipseq_eapca", "skipseq_sax"}


def test_results_struct_tie_order():
    r = search.Results(3)
    for d, i in ((2.0, 9), (1.0, 4), (2.0, 3), (2.0, 1), (5.0, 0)):
        r.offer(d, i)
    assert r.d == [1.0, 2.0, 2.0] and r.id == [4, 1, 3]
