"""Parity at the benchmark's full size, in the launch configuration bench.py
times: 10,000,000 random-walk series of length 256, 300 queries (100 each at
1 %, 5 % and 10 % noise), k = 10, w = 16, leaves of 10,000, l_max = 4, one
call for the whole batch.  The oracle computes a sample of the queries (its
FP64 brute force over all 10M series), spread over the three noise levels;
the plain path and the precision form must both match it on every sampled
query, and the two forms' id lists must agree on every query.
"""
import numpy as np
import pytest

from oracle import brute
from paper_2212_13297_amd import datagen as G

from parity import check_knn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_full_size_sampled_parity():
    from paper_2212_13297_amd import hs
    N, n, k = 10_000_000, 256, 10
    print(f"[fullsize] generating {N} x {n}", flush=True)
    x = G.random_walks(N, n)
    q, _, pct = G.workload(x, [1, 5, 10], 100)
    xt = torch.from_numpy(x).to(DEV)
    idx = hs.Index(xt, hs.Params(w=16, leaf_size=10_000, l_max=4, seed_rows=256))
    torch.cuda.synchronize()
    del xt
    torch.cuda.empty_cache()
    qt = torch.from_numpy(q).to(DEV)
    print("[fullsize] plain batch", flush=True)
    ids, d2, st = idx.knn(qt, k, stats=True)
    torch.cuda.synchronize()
    ids, d2 = ids.cpu().numpy(), d2.cpu().numpy()
    print("[fullsize] precision-form batch", flush=True)
    idx.build_shadow(hs.HS_SHADOW_BF16)
    mids, md2, merr = idx.knn_mixed(qt, k)
    torch.cuda.synchronize()
    mids, md2, merr = mids.cpu().numpy(), md2.cpu().numpy(), merr.cpu().numpy()
    sel = np.concatenate([np.where(pct == p)[0][::20] for p in (1, 5, 10)])  # 15 queries
    print(f"[fullsize] oracle on {len(sel)} queries", flush=True)
    oids, od = brute.knn(x, q[sel], k)
    full_o = np.zeros((len(q), k), np.int64)
    full_d = np.zeros((len(q), k))
    full_o[sel], full_d[sel] = oids, od
    check_knn(x, q, k, ids, d2, full_o, full_d, qsel=sel)
    check_knn(x, q, k, mids, md2, full_o, full_d, qsel=sel)
    d64 = brute.pair_dist(x, q, np.repeat(sel.astype(np.int32), k), mids[sel].reshape(-1)).reshape(len(sel), k)
    assert np.all(np.abs(md2[sel].astype(np.float64) - d64) <= merr[sel])
    # the two forms agree on every query (ties within 1e-6 aside, none expected here)
    same = (ids == mids).all(axis=1)
    assert same.mean() > 0.99, f"plain and precision id lists differ on {np.sum(~same)} queries"
    assert int(st["rounds"].max().item()) >= 1
    idx.close()
