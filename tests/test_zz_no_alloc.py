"""The no-allocation entry point (hs_knn_exact_noalloc) against hs_knn_exact.

Through the C ABI, on the same index and queries: ids, distances and error
bounds bit for bit, and the FP64 oracle's k-NN; two calls in a row, the
second with fewer queries and a smaller k (the static array keeps the first
call's contents); a batch whose candidates overflow the array's smaller
candidate list (overflow rounds, same results); and the size limit.
"""
import numpy as np
import pytest

from paper_2212_13297_amd import datagen as G

from parity import check_err, check_knn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def hs_mod():
    from paper_2212_13297_amd import hs
    return hs


def noalloc(idx, qt, k, stats=False):
    hs = hs_mod()
    Q = qt.shape[0]
    ids = torch.full((Q, k), -7, dtype=torch.int64, device=DEV)
    d2 = torch.full((Q, k), -1.0, dtype=torch.float32, device=DEV)
    err = torch.full((Q, k), -1.0, dtype=torch.float64, device=DEV)
    st = torch.zeros((Q, 8), dtype=torch.int64, device=DEV) if stats else None
    print(f"[noalloc] Q={Q} k={k}", flush=True)
    hs.hs_knn_exact_noalloc(idx.h, qt.data_ptr(), Q, k, ids.data_ptr(), d2.data_ptr(), err.data_ptr(),
                            st.data_ptr() if st is not None else None,
                            int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    out = (ids.cpu().numpy(), d2.cpu().numpy(), err.cpu().numpy())
    return out + ((st.cpu().numpy(),) if stats else ())


def with_workspace(idx, qt, k):
    print(f"[knn] Q={qt.shape[0]} k={k}", flush=True)
    ids, d2, err = idx.knn(qt, k, err=True)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d2.cpu().numpy(), err.cpu().numpy()


def same(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
    assert np.array_equal(a[2], b[2])


def test_noalloc_equals_workspace_entry_point_two_calls():
    hs = hs_mod()
    x = G.random_walks(30_000, 256, coll=91)
    q, _, _ = G.workload(x, [1, 5, 10], 6, coll=91)
    q = np.concatenate([q, G.ood_queries(3, 256, coll=91)])
    idx = hs.Index(torch.from_numpy(x).to(DEV), hs.Params(w=16, leaf_size=1000, l_max=2))
    qt = torch.from_numpy(q).to(DEV)
    # first call: 21 queries, k = 10
    a = noalloc(idx, qt, 10)
    b = with_workspace(idx, qt, 10)
    same(a, b)
    check_knn(x, q, 10, a[0], a[1])
    check_err(x, q, a[0], a[1], a[2])
    # second call: fewer queries and a smaller k, on the array the first left behind
    q2 = q[5:12].copy()
    qt2 = torch.from_numpy(q2).to(DEV)
    a2 = noalloc(idx, qt2, 4)
    b2 = with_workspace(idx, qt2, 4)
    same(a2, b2)
    check_knn(x, q2, 4, a2[0], a2[1])
    idx.close()


def test_noalloc_candidate_overflow_and_size_limit():
    hs = hs_mod()
    # white-noise queries keep nearly every series as a candidate: 64 queries
    # x 200,000 series do not fit the array's candidate list, so queries take
    # the overflow rounds; the results still equal hs_knn_exact's
    N, n, k = 200_000, 256, 10
    x = G.random_walks(N, n, coll=92)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([92, 1])))
    noise = g.standard_normal((64, n))
    noise = ((noise - noise.mean(1, keepdims=True)) / noise.std(1, keepdims=True)).astype(np.float32)
    q = np.concatenate([noise, G.workload(x, [10], 4, coll=92)[0]])
    idx = hs.Index(torch.from_numpy(x).to(DEV), hs.Params(w=16, leaf_size=2000, l_max=1, cand_per_query=2 * N))
    qt = torch.from_numpy(q).to(DEV)
    a = noalloc(idx, qt, k, stats=True)
    b = with_workspace(idx, qt, k)
    same(a[:3], b)
    rounds = a[3][:, 5]
    print(f"[noalloc] rounds > 1 on {int((rounds > 1).sum())} of {len(q)} queries", flush=True)
    assert rounds.max() >= 2
    sel = np.arange(0, len(q), 5)
    check_knn(x, q, k, a[0], a[1], qsel=sel)
    # a batch whose per-query tables alone exceed the array is refused before
    # any device work, and the entry point still answers afterwards
    big = torch.zeros((4000, n), dtype=torch.float32, device=DEV)
    ids = torch.empty((4000, k), dtype=torch.int64, device=DEV)
    d2 = torch.empty((4000, k), dtype=torch.float32, device=DEV)
    with pytest.raises(hs.HSError) as e:
        hs.hs_knn_exact_noalloc(idx.h, big.data_ptr(), 4000, k, ids.data_ptr(), d2.data_ptr(), None, None,
                                int(torch.cuda.current_stream().cuda_stream))
    assert e.value.code == hs.HS_EINVAL
    a3 = noalloc(idx, qt[:3].contiguous(), 3)
    same(a3, with_workspace(idx, qt[:3].contiguous(), 3))
    idx.close()
