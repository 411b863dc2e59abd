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


@pytest.mark.parametrize("tau,l_max,k", [(1, 1, 1), (50, 0, 3), (50, 3, 5), (200, 1, 10), (4000, 2, 4)])
def test_tree_search_picks_the_flat_leaves(data, tau, l_max, k):
    # Sec. 3.4's priority queue over the tree (internal synopses from their
    # children's) seeds from and keeps exactly the leaves that sorting every
    # leaf's own LB_EAPCA gives, and both equal brute force.
    x, q = data
    t = search.TreeIndex(x, 16, tau)
    ids, d2 = brute.knn(x, q, k)
    for i in range(len(q)):
        s1, s2 = {}, {}
        a = search.exact_knn(t, q[i], k, l_max=l_max, stats=s1)
        b = search.exact_knn_tree(t, q[i], k, l_max=l_max, stats=s2)
        assert s1["seeded"] == s2["seeded"]
        assert s1["kept"] == s2["kept"]
        np.testing.assert_array_equal(b[0], ids[i])
        np.testing.assert_array_equal(b[1], d2[i])
        np.testing.assert_array_equal(a[0], b[0])


def test_tree_bounds_are_monotone_down_the_tree(data):
    # A parent's synopsis (the union of its children's) contains every
    # descendant's box, so its LB_EAPCA never exceeds theirs: the largest bound
    # over a leaf's ancestors is the leaf's own, bit for bit.
    from oracle import summaries as S
    x, q = data
    t = search.TreeIndex(x, 16, 50)
    assert len(t.nodes) == 2 * len(t.leaves) - 1
    # the root's synopsis is the one over every series
    mu, sd = S.segment_stats(x, t.ends)
    np.testing.assert_array_equal(t.node_syn[0], S.synopsis(mu, sd))
    parent = {}
    for v, node in enumerate(t.nodes):
        if node["children"] is not None:
            for c in node["children"]:
                parent[c] = v
                lo_ok = t.node_syn[v][:, [0, 2]] <= t.node_syn[c][:, [0, 2]]
                hi_ok = t.node_syn[v][:, [1, 3]] >= t.node_syn[c][:, [1, 3]]
                assert lo_ok.all() and hi_ok.all()
    for qi in range(len(q)):
        mq, sq = S.segment_stats(q[qi].astype(np.float64), t.ends)
        lb = [float(S.lb_eapca(mq, sq, syn, t.ends)) for syn in t.node_syn]
        for v, node in enumerate(t.nodes):
            if node["children"] is None:
                anc, u = [], v
                while u in parent:
                    u = parent[u]
                    anc.append(lb[u])
                assert max(anc + [lb[v]]) == lb[v]
