"""GPU parity of the precision form (hs_build_shadow / hs_knn_mixed).

The precision form must return the oracle's exact k-NN (same acceptance as
the plain path), every result's distance must lie within the error bound the
library reports beside it (and that bound within 1e-5 relative), and its ids
and distances must equal the plain path's on the same index (both forms key
their results by the same compensated distance).  Covers bf16 and fp16
copies, one, two and four K-blocks (n = 256, 320 and 1024), w = 32 with
k = 100 and out-of-distribution queries (the long-series configuration),
several k, q-group counts (Q below and above 128), the overflow fallback,
and argument errors.
"""
import numpy as np
import pytest

from oracle import precision as P
from paper_2212_13297_amd import datagen as G

from parity import check_err, check_knn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def hs_mod():
    from paper_2212_13297_amd import hs
    return hs


def make_index(x, kind, **kw):
    hs = hs_mod()
    print(f"[build] N={x.shape[0]} n={x.shape[1]} kind={kind} {kw}", flush=True)
    idx = hs.Index(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), hs.Params(**kw))
    if kind:
        idx.build_shadow(kind)
    torch.cuda.synchronize()
    return idx


def knn_mixed(idx, q, k, **kw):
    print(f"[knn_mixed] Q={q.shape[0]} k={k}", flush=True)
    out = idx.knn_mixed(torch.from_numpy(np.ascontiguousarray(q)).to(DEV), k, **kw)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() if hasattr(o, "cpu") else {f: v.cpu().numpy() for f, v in o.items()}
                 for o in out)


def knn_plain(idx, q, k):
    print(f"[knn] Q={q.shape[0]} k={k}", flush=True)
    ids, d2 = idx.knn(torch.from_numpy(np.ascontiguousarray(q)).to(DEV), k)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d2.cpu().numpy()


def workload(N, n, coll, per_level=3, ood=2):
    x = G.random_walks(N, n, coll=coll)
    q, _, _ = G.workload(x, [1, 5, 10], per_level, coll=coll)
    if ood:
        q = np.concatenate([q, G.ood_queries(ood, n, coll=coll)])
    return x, q


@pytest.mark.parametrize("kind", [P.BF16, P.FP16])
def test_shadow_copy_against_oracle(kind):
    N, n = 5003, 320
    x = G.random_walks(N, n, coll=41)
    idx = make_index(x, kind, w=16, leaf_size=500)
    rows, ids, _, _, _ = idx.layout()
    rows = rows.cpu().numpy()
    stride = idx.info.row_stride
    sh = idx.shadow.cpu().numpy()
    pad = 32  # zero rows after the copy
    low_bits = sh[:N * stride * 2].view(np.uint16).reshape(N, stride)
    assert not np.any(sh[N * stride * 2:(N + pad) * stride * 2])
    norms = sh[((N + pad) * stride * 2 + 255) // 256 * 256:][:N * 16].view(np.float32).reshape(N, 4)
    if kind == P.BF16:
        low = (low_bits.astype(np.uint32) << 16).view(np.float32)
    else:
        low = low_bits.view(np.float16).astype(np.float32)
    np.testing.assert_array_equal(low, P.round_low(rows, kind))
    xn = np.sum(low.astype(np.float64) ** 2, axis=1)
    eps = np.sqrt(np.sum((rows.astype(np.float64) - low.astype(np.float64)) ** 2, axis=1))
    assert np.all(norms[:, 2] <= xn) and np.all(norms[:, 2] >= xn * (1 - 1e-6))
    assert np.all(norms[:, 1] >= eps) and np.all(norms[:, 1] <= eps * (1 + 1e-6) + 1e-37)
    # the augmented unit (a*, ebar) of the bounding pass, two low-precision values
    au = norms[:, 3].view(np.uint32)
    if kind == P.BF16:
        dec = lambda b: (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        dec = lambda b: b.astype(np.uint16).view(np.float16).astype(np.float64)
    a_st, eb = dec(au & 0xFFFF), dec(au >> 16)
    assert np.all(eb >= norms[:, 1].astype(np.float64))
    # beta = ((1 - g) xn - eps^2) / 2 - 3u (xn + eps^2) from the stored xn and eps,
    # rounded down to float32 (g: accumulation factor of `stride` additions)
    u2 = 2.0 ** -23
    g = stride * u2 / (1.0 - stride * u2) + 2.0 ** -40
    xs, es = norms[:, 2].astype(np.float64), norms[:, 1].astype(np.float64)
    beta = 0.5 * ((1.0 - g) * xs - es * es) - 3.0 * 2.0 ** -24 * (xs + es * es)
    b32 = norms[:, 0]
    assert np.all(b32.astype(np.float64) <= beta)
    assert np.all(np.nextafter(b32, np.float32(np.inf)).astype(np.float64) > beta)
    # a* >= -B0 + g2 (||x~||^2 / 2 + |a*| + ebar^2 / 2), B0 from the stored values,
    # g2 the accumulation factor of stride + 2 products
    g2 = (stride + 2) * u2 / (1.0 - (stride + 2) * u2)
    B0 = 0.5 * (xs - es * es)
    assert np.all(a_st >= -B0 + g2 * (0.5 * xn + np.abs(a_st) + 0.5 * eb * eb))


# N, n, w, k, leaf, l_max, per_level, kind
CASES = [
    (20000, 256, 16, 10, 1000, 2, 3, P.BF16),
    (20000, 256, 16, 10, 1000, 2, 3, P.FP16),
    (9001, 320, 16, 5, 700, 1, 2, P.BF16),      # two K-blocks, ragged tiles
    (12000, 128, 8, 1, 500, 4, 3, P.FP16),
    (30000, 256, 16, 50, 2000, 4, 2, P.BF16),
    # long series: n = 1024 (four K-blocks), w = 32, k = 100, ood queries
    (20000, 1024, 32, 100, 1000, 2, 2, P.BF16),
    (20000, 1024, 32, 100, 1000, 2, 2, P.FP16),
]


@pytest.mark.parametrize("N,n,w,k,leaf,lmax,per,kind", CASES)
def test_mixed_parity(N, n, w, k, leaf, lmax, per, kind):
    x, q = workload(N, n, coll=50 + n, per_level=per, ood=4 if n == 1024 else 2)
    idx = make_index(x, kind, w=w, leaf_size=leaf, l_max=lmax)
    ids, d2, err, st = knn_mixed(idx, q, k, stats=True)
    print(f"[case] rows bounded {st['rows_bounded'].mean():.0f}, candidates {st['candidates'].mean():.1f}, "
          f"refined {st['rows_refined'].mean():.1f}", flush=True)
    oids, od = check_knn(x, q, k, ids, d2)
    rel = check_err(x, q, ids, d2, err)
    assert rel < 5e-7
    pids, pd2 = knn_plain(idx, q, k)
    check_knn(x, q, k, pids, pd2, oids, od)
    # the plain path's ids and distances, bit for bit: both are the exact
    # top-k by the same compensated distance
    assert np.array_equal(pids, ids)
    assert np.array_equal(pd2.view(np.uint32), d2.view(np.uint32))


@pytest.mark.parametrize("N,n,w,k,kind,fracs", [(30000, 256, 16, 10, P.BF16, (0.0, 0.3, 0.97)),
                                                 (12000, 1024, 32, 100, P.FP16, (0.6,))])
def test_mixed_partial_copy(N, n, w, k, kind, fracs):
    # A low-precision copy of only the first whole parts (shadow_rows): the
    # matrix-core bound covers those series, LB_SAX the rest, one candidate
    # list, the compensated refine; ids and distances equal the plain path's
    # and the oracle's.  From no series at all to nearly all of them.
    hs = hs_mod()
    x, q = workload(N, n, coll=90 + n, per_level=3, ood=3)
    idx = make_index(x, 0, w=w, leaf_size=700, l_max=2)
    pids, pd2 = knn_plain(idx, q, k)
    oids, od = check_knn(x, q, k, pids, pd2)
    for f in fracs:
        rows = int(f * N)
        idx.build_shadow(kind, shadow_rows=rows)
        covered = hs.hs_shadow_bytes(idx.h, kind, rows)
        print(f"[partial] shadow_rows {rows}: {covered} bytes", flush=True)
        ids, d2, err, st = knn_mixed(idx, q, k, stats=True)
        assert np.array_equal(ids, pids)
        assert np.array_equal(d2.view(np.uint32), pd2.view(np.uint32))
        check_knn(x, q, k, ids, d2, oids, od)
        check_err(x, q, ids, d2, err)
        # the copy's series are bounded on the matrix cores, the others by LB_SAX
        assert np.all(st["rows_filtered"] + st["rows_bounded"] > 0)
        assert np.all(st["bound_pairs"] >= st["rows_bounded"])
        if rows == 0:
            assert st["rows_bounded"].sum() == 0
        else:
            assert st["rows_bounded"].sum() > 0
    idx.close()


def test_mixed_many_query_groups():
    # Q = 300: three q-groups of 128, the last one partial
    x = G.random_walks(15000, 256, coll=61)
    q, _, _ = G.workload(x, [1, 5, 10], 100, coll=61)
    idx = make_index(x, P.BF16, w=16, leaf_size=1000, l_max=2)
    ids, d2, err = knn_mixed(idx, q, 10)
    sel = np.arange(0, 300, 7)
    check_knn(x, q, 10, ids, d2, qsel=sel)
    check_err(x[:, :], q[sel], ids[sel], d2[sel], err[sel])


def test_mixed_single_query_and_batch_independence():
    x, q = workload(12000, 256, coll=62)
    idx = make_index(x, P.BF16, w=16, leaf_size=800, l_max=1)
    ids, d2, err = knn_mixed(idx, q, 7)
    for i in (0, 5, len(q) - 1):
        i1, d1, e1 = knn_mixed(idx, q[i:i + 1], 7)
        assert np.array_equal(i1[0], ids[i]) and np.array_equal(d1[0], d2[i])


def test_mixed_overflow_fallback():
    # tiny candidate capacity: survivors spill, the queries are answered by
    # the fused fallback with the compensated distance, same results
    x, q = workload(16000, 256, coll=63)
    idx = make_index(x, P.BF16, w=16, leaf_size=1000, l_max=1, cand_per_query=16)
    ids, d2, err, st = knn_mixed(idx, q, 10, stats=True)
    assert int(st["rounds"].max()) >= 2
    check_knn(x, q, 10, ids, d2)
    check_err(x, q, ids, d2, err)


def test_mixed_without_seed():
    # l_max = 0: BSF_k starts at infinity, every pair survives the bound and
    # the candidate list overflows into the fallback
    x, q = workload(6000, 128, coll=64, per_level=1, ood=1)
    idx = make_index(x, P.FP16, w=8, leaf_size=400, l_max=0)
    ids, d2, err = knn_mixed(idx, q, 3)
    check_knn(x, q, 3, ids, d2)
    check_err(x, q, ids, d2, err)


def test_mixed_white_noise_queries():
    # White-noise queries (z-normalised) are far from every series: LB_SAX
    # keeps nearly all of them, the matrix-core bound about one in 120.  The
    # results, their error bounds and the plain form's id lists still agree.
    N, n, k = 200_000, 256, 10
    x = G.random_walks(N, n, coll=78)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([78, 1])))
    noise = g.standard_normal((64, n))
    noise = ((noise - noise.mean(1, keepdims=True)) / noise.std(1, keepdims=True)).astype(np.float32)
    q = np.concatenate([noise, G.workload(x, [10], 8, coll=78)[0]])
    idx = make_index(x, P.BF16, w=16, leaf_size=2000, l_max=1, cand_per_query=2 * N)
    ids, d2, err, st = knn_mixed(idx, q, k, stats=True)
    # a query whose candidates spread over hundreds of wavefronts can fill its
    # result pool with their flushed top-k lists and take the fallback round
    print(f"[white noise, precision form] candidates {int(st['candidates'].sum())}, "
          f"fallback rounds on {int((st['rounds'] > 1).sum())} queries", flush=True)
    check_knn(x, q, k, ids, d2)
    check_err(x, q, ids, d2, err)
    pids, _ = knn_plain(idx, q, k)
    assert np.array_equal(ids, pids)
    idx.close()


def test_mixed_errors():
    hs = hs_mod()
    x = G.random_walks(3000, 64, coll=65)
    idx = make_index(x, 0, w=8, leaf_size=300)
    q = torch.from_numpy(x[:2].copy()).to(DEV)
    with pytest.raises(hs.HSError):
        idx.knn_mixed(q, 3)  # no low-precision copy
    with pytest.raises(hs.HSError):
        idx.build_shadow(7)  # unknown kind
    big = make_index((x * 1e5).astype(np.float32), 0, w=8, leaf_size=300)
    with pytest.raises(hs.HSError):
        big.build_shadow(hs.HS_SHADOW_FP16)  # beyond the fp16 range
    big.build_shadow(hs.HS_SHADOW_BF16)      # bf16 covers the float32 range
    idx.build_shadow(hs.HS_SHADOW_FP16)
    with pytest.raises(hs.HSError):
        idx.knn_mixed((q * 1e6).contiguous(), 3)  # query beyond the fp16 range
