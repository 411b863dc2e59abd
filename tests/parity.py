"""Comparison of GPU k-NN results against the FP64 oracle (test helper).

Acceptance (per query): the GPU id list is sorted by (d, id), has no repeats,
and every reported distance is within 1e-5 relative of the FP64 distance of
the same pair; the GPU id set equals the oracle's, except for ids whose FP64
distance lies in the tie band |d64 - d64_k| <= 1e-6 * d64_k around the
oracle's k-th distance (either side may hold a different member of the band).
"""
import numpy as np

from oracle import brute

REL_D = 1e-5
TIE = 1e-6


def check_knn(x, q, k, ids, d2, oids=None, od=None, qsel=None):
    """Raise AssertionError on any violation.  qsel: indices of queries to check."""
    ids = np.asarray(ids)
    d2 = np.asarray(d2, dtype=np.float64)
    Q = q.shape[0]
    qsel = np.arange(Q) if qsel is None else np.asarray(qsel)
    if oids is None:
        oids, od = brute.knn(x, q[qsel], k)
    else:
        oids, od = oids[qsel], od[qsel]
    for j, i in enumerate(qsel):
        g = ids[i]
        assert len(set(g.tolist())) == k, f"query {i}: repeated ids {g}"
        assert np.all(g >= 0) and np.all(g < x.shape[0]), f"query {i}: id out of range"
        assert np.all(np.diff(d2[i]) >= 0), f"query {i}: distances not ascending"
        d64 = brute.pair_dist(x, q, np.full(k, i, np.int32), g)
        err = np.abs(d2[i] - d64)
        assert np.all(err <= REL_D * d64 + 1e-30), f"query {i}: distance error {np.max(err / np.maximum(d64, 1e-30))}"
        dk = od[j, -1]
        band = TIE * dk
        only_g = set(g.tolist()) - set(oids[j].tolist())
        only_o = set(oids[j].tolist()) - set(g.tolist())
        for a in only_g:
            da = d64[list(g).index(a)]
            assert abs(da - dk) <= band, f"query {i}: id {a} (d={da}) not in oracle top-{k} (kth={dk})"
        for a in only_o:
            da = od[j][list(oids[j]).index(a)]
            assert abs(da - dk) <= band, f"query {i}: oracle id {a} (d={da}) missing (kth={dk})"
    return oids, od


def check_err(x, q, ids, d2, err):
    """|d2 - d64| <= err <= 1e-5 d64 for every result; returns the largest
    measured relative error."""
    ids = np.asarray(ids)
    Q, k = ids.shape
    qi = np.repeat(np.arange(Q, dtype=np.int32), k)
    d64 = brute.pair_dist(x, q, qi, ids.reshape(-1)).reshape(Q, k)
    meas = np.abs(np.asarray(d2, dtype=np.float64) - d64)
    err = np.asarray(err, dtype=np.float64)
    assert np.all(meas <= err), f"measured error above the reported bound: {np.max(meas - err)}"
    assert np.all(err <= REL_D * d64), "reported bound above 1e-5 relative"
    return float(np.max(meas / np.maximum(d64, 1e-30)))
