"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Covers the index build (stored copy, id map, iSAX words, leaf synopses), exact
k-NN at several shapes (ragged n, several w, k, leaf sizes and seed sizes,
noise levels 1/5/10 % and out-of-dataset queries), the access paths, edge
cases, determinism and argument errors.
"""
import math

import numpy as np
import pytest

from oracle import brute
from oracle import summaries as S
from paper_2212_13297_amd import datagen as G

from parity import check_err, check_knn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def hs_mod():
    from paper_2212_13297_amd import hs
    return hs


def make_index(x, **kw):
    hs = hs_mod()
    print(f"[build] N={x.shape[0]} n={x.shape[1]} {kw}", flush=True)
    return hs.Index(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), hs.Params(**kw))


def run_knn(idx, q, k, **kw):
    print(f"[knn] Q={q.shape[0]} k={k}", flush=True)
    out = idx.knn(torch.from_numpy(np.ascontiguousarray(q)).to(DEV), k, **kw)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() if hasattr(o, "cpu") else o for o in out)


def workload(N, n, coll, per_level=3, ood=2):
    x = G.random_walks(N, n, coll=coll)
    q, _, _ = G.workload(x, [1, 5, 10], per_level, coll=coll)
    if ood:
        q = np.concatenate([q, G.ood_queries(ood, n, coll=coll)])
    return x, q


# ------------------------------------------------------------------ build

def test_build_summaries_against_oracle():
    N, n, w, tau = 30011, 256, 16, 700
    x = G.random_walks(N, n, coll=11)
    idx = make_index(x, w=w, leaf_size=tau)
    rows, ids, words, ls, env = idx.layout()
    rows, ids, words = rows.cpu().numpy(), ids.cpu().numpy().astype(np.int64), words.cpu().numpy()
    info = idx.info
    assert info.n_leaves == len(ls) - 1 and ls[0] == 0 and ls[-1] == N
    assert np.all(np.diff(ls) > 0)
    # the id map is a permutation and the stored rows are the inputs, zero padded
    assert np.array_equal(np.sort(ids), np.arange(N))
    assert np.array_equal(rows[:, :n], x[ids])
    assert np.all(rows[:, n:] == 0)
    sizes = np.diff(ls)
    assert sizes.max() <= tau
    # chunks: each leaf cut into 64-series chunks from its first series; the
    # chunk envelopes contain their members' FP64 statistics
    from paper_2212_13297_amd import hs
    cs, cenv = hs.hs_get_chunks(idx.h, info)
    expect = np.concatenate([np.arange(a, b, 64) for a, b in zip(ls[:-1], ls[1:])] + [[N]])
    assert np.array_equal(cs, expect)
    mu_c, sd_c = S.segment_stats(x[ids], S.equal_segmentation(n, w))
    for i, (a, b) in enumerate(zip(cs[:-1], cs[1:])):
        e = cenv[i].astype(np.float64)
        assert np.all(mu_c[a:b] >= e[:, 0]) and np.all(mu_c[a:b] <= e[:, 1])
        assert np.all(sd_c[a:b] >= e[:, 2]) and np.all(sd_c[a:b] <= e[:, 3])
    # iSAX words: equal to the oracle's except where the PAA lies within 1e-6 of a breakpoint
    beta = S.breakpoints(256)
    paa = S.paa(x[ids], w)
    ow = S.sax_word(paa, beta).astype(np.int64)
    gw = words[:, :w].astype(np.int64)
    diff = np.nonzero(ow != gw)
    for r, c in zip(*diff):
        near = np.min(np.abs(beta[1:-1] - paa[r, c]))
        assert near < 1e-6 and abs(ow[r, c] - gw[r, c]) == 1, (r, c, paa[r, c], ow[r, c], gw[r, c])
    # leaf synopses contain every member's FP64 segment statistics
    ends = S.equal_segmentation(n, w)
    mu, sd = S.segment_stats(x[ids], ends)
    for i, (a, b) in enumerate(zip(ls[:-1], ls[1:])):
        e = env[i].astype(np.float64)
        assert np.all(mu[a:b] >= e[:, 0]) and np.all(mu[a:b] <= e[:, 1])
        assert np.all(sd[a:b] >= e[:, 2]) and np.all(sd[a:b] <= e[:, 3])
        syn = S.synopsis(mu[a:b], sd[a:b])
        assert np.all(np.abs(syn - e) <= 1e-6 * (1 + np.abs(syn)))   # and are tight
    # deviation codes: the width covers the largest std over 256 codes with at
    # most 16 significant bits (so c h is exact in float32), every code's
    # interval contains its FP64 std, and the codes equal the oracle's except
    # where the std lies within 1e-9 relative of a code boundary
    codes, h = idx.sigma_codes()
    codes = codes.cpu().numpy()
    assert h > 0 and 256 * h > sd.max() and 128 * h <= sd.max() * (1 + 1e-5)
    m, e = np.frexp(h)
    assert (m * 65536) == np.floor(m * 65536)
    gc = codes[:, :w].astype(np.float64)
    assert np.all(codes[:, w:] == 0)
    assert np.all(gc * h <= sd) and np.all(sd < (gc + 1) * h)
    oc = S.sigma_codes(sd, h).astype(np.float64)
    for r, c in zip(*np.nonzero(oc != gc)):
        assert abs(sd[r, c] / h - round(sd[r, c] / h)) < 1e-9 * (1 + sd[r, c] / h), (r, c, sd[r, c], gc[r, c])
    idx.close()


@pytest.mark.parametrize("N,n,w,tau,dup", [(30_011, 256, 16, 700, 0), (3_000, 64, 8, 1, 0), (12_000, 64, 64, 50, 0),
                                           (9_000, 200, 5, 333, 2_000), (70_000, 128, 16, 10_000, 0)])
def test_device_partition_equals_host_partition(N, n, w, tau, dup):
    # The level-by-level device partition and the recursive host partition
    # make the same leaves and store the series in the same order (same
    # float32 statistics, same FP64 thresholds and scores); hence the same
    # words, envelopes and chunk tables.  Cases: ragged N, one series per
    # leaf, w = 64 (its scratch outside the rows' area), w = 5 (2w = 10
    # statistics), thousands of exact duplicates (unsplittable nodes), and
    # leaves of 10,000.
    hs = hs_mod()
    x = G.random_walks(N, n, coll=40 + w).copy()
    if dup:
        x[np.arange(3, N, 4)[:dup]] = x[1]
    a = make_index(x, w=w, leaf_size=tau)
    b = make_index(x, w=w, leaf_size=tau, build_flags=hs.HS_BUILD_HOST_PARTITION)
    ra, ia, wa, la, ea = a.layout()
    rb, ib, wb, lb, eb = b.layout()
    assert np.array_equal(la, lb)
    assert torch.equal(ia, ib) and torch.equal(ra, rb) and torch.equal(wa, wb)
    assert np.array_equal(ea, eb)
    ca, cea = hs.hs_get_chunks(a.h, a.info)
    cb, ceb = hs.hs_get_chunks(b.h, b.info)
    assert np.array_equal(ca, cb) and np.array_equal(cea, ceb)
    sizes = np.diff(la)
    print(f"[partition] {len(la) - 1} leaves, largest {sizes.max()}, smallest {sizes.min()}", flush=True)
    if not dup:
        assert sizes.max() <= tau
    a.close()
    b.close()


def test_streaming_build_equals_one_call_build():
    # The same index from uneven row chunks given twice (statistics, then
    # rows) as from one call; chunk order and turn are enforced; NaN in a
    # chunk is reported by the partition step.
    hs = hs_mod()
    N, n = 25_013, 256
    x = G.random_walks(N, n, coll=33)
    xt = torch.from_numpy(x).to(DEV)
    a = hs.Index(xt, hs.Params(w=16, leaf_size=600))
    sizes = [7001, 1, 9000, N - 16002]
    starts = np.concatenate([[0], np.cumsum(sizes)])
    calls = []

    def chunk(r0):
        i = int(np.searchsorted(starts, r0))
        calls.append(r0)
        return xt[r0:r0 + sizes[i]].contiguous()

    b = hs.Index.from_chunks(chunk, N, n, hs.Params(w=16, leaf_size=600))
    assert calls == list(starts[:-1]) * 2
    ra, ia, wa, la, ea = a.layout()
    rb, ib, wb, lb, eb = b.layout()
    assert np.array_equal(la, lb) and np.array_equal(ea, eb)
    assert torch.equal(ia, ib) and torch.equal(ra, rb) and torch.equal(wa, wb)
    q = G.workload(x, [1, 10], 3, coll=33)[0]
    r1 = run_knn(a, q, 10)
    r2 = run_knn(b, q, 10)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])
    check_knn(x, q, 10, r2[0], r2[1])
    # steps out of turn and chunks out of order are refused
    p = hs.Params(w=16, leaf_size=600).c(n)
    nb = hs.hs_index_bytes(N, p)
    mem = torch.empty(nb, dtype=torch.uint8, device=DEV)
    st = int(torch.cuda.current_stream().cuda_stream)
    h = hs.hs_build_begin(N, p, mem.data_ptr(), nb, st)
    with pytest.raises(hs.HSError):
        hs.hs_build_add_stats(h, xt.data_ptr(), 5, 10)       # must start at row 0
    with pytest.raises(hs.HSError):
        hs.hs_build_partition(h)                             # statistics of all rows first
    with pytest.raises(hs.HSError):
        hs.hs_build_add_rows(h, xt.data_ptr(), 0, 10)        # rows after the partition
    hs.hs_build_abort(h)
    bad = xt.clone()
    bad[20_000, 7] = float("nan")
    h = hs.hs_build_begin(N, p, mem.data_ptr(), nb, st)
    hs.hs_build_add_stats(h, bad.data_ptr(), 0, N)
    with pytest.raises(hs.HSError) as e:
        hs.hs_build_partition(h)
    assert e.value.code == hs.HS_EINVAL
    hs.hs_build_abort(h)
    a.close()
    b.close()


# ----------------------------------------------------------------- parity

CASES = [
    # N, n, w, tau, l_max, k
    (100_000, 256, 16, 1000, 1, 1),      # the small plain configuration
    (12_345, 200, 8, 333, 1, 7),         # n not a multiple of 64: padded rows
    (20_000, 128, 16, 1000, 1, 100),     # k = 100
    (20_000, 1024, 32, 500, 2, 10),      # long series, w = 32
    (15_000, 512, 16, 400, 1, 10),       # two chunks per quarter in the refine's chunk order
    (9_000, 256, 16, 100, 0, 10),        # no seed leaves
    (9_000, 256, 16, 50, 5, 3),          # several seed leaves, small leaves
    (5_000, 64, 4, 5_000, 1, 20),        # a single leaf
    (8_000, 320, 20, 400, 1, 5),         # w = 20: two-block words with 12 padding segments
    (6_000, 384, 48, 300, 2, 10),        # w = 48: three-block words
    (4_000, 256, 64, 500, 1, 4),         # w = 64: four-block words, 4 points per segment
]


@pytest.mark.parametrize("n,w", [(256, 16), (1024, 32)])
def test_distance_independent_of_path(n, w):
    # A pair's float32 distance is the same whether the seed step (natural
    # chunk order) or the refine (chunks read in LB_SAX order, distance of an
    # admitted series summed again in natural order) produced it: without
    # seed leaves every result comes from the refine.
    x, q = workload(6000, n, coll=n + w, per_level=4)
    a = make_index(x, w=w, leaf_size=150, l_max=0)
    b = make_index(x, w=w, leaf_size=150, l_max=6)
    ia, da = run_knn(a, q, 10)
    ib, db = run_knn(b, q, 10)
    check_knn(x, q, 10, ia, da)
    common = 0
    for i in range(q.shape[0]):
        mb = dict(zip(ib[i].tolist(), db[i].tolist()))
        for j, d in zip(ia[i].tolist(), da[i].tolist()):
            if j in mb:
                assert np.float32(d).view(np.uint32) == np.float32(mb[j]).view(np.uint32), (i, j, d, mb[j])
                common += 1
    assert common >= 5 * q.shape[0]
    a.close()
    b.close()


def test_long_candidate_list():
    # White-noise queries (z-normalised) keep nearly every series as a
    # candidate: the refine then deals its list out in segments from a counter
    # (a list of at least two segments per wavefront) rather than one range
    # each.
    N, n, k = 200_000, 256, 10
    x = G.random_walks(N, n, coll=77)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([77, 1])))
    noise = g.standard_normal((64, n))
    noise = ((noise - noise.mean(1, keepdims=True)) / noise.std(1, keepdims=True)).astype(np.float32)
    q = np.concatenate([noise, G.workload(x, [10], 8, coll=77)[0]])
    idx = make_index(x, w=16, leaf_size=2000, l_max=1, cand_per_query=2 * N)
    ids, d2, st = run_knn(idx, q, k, stats=True)
    cands = int(st["candidates"].sum().item())
    print(f"[long list] candidates {cands}", flush=True)
    assert cands >= 2 * 4096 * 512
    assert int(st["rounds"].max().item()) == 1  # no overflow fallback
    check_knn(x, q, k, ids, d2)
    idx.close()


@pytest.mark.parametrize("N,n,w,tau,l_max,k", CASES)
def test_knn_parity(N, n, w, tau, l_max, k):
    x, q = workload(N, n, coll=N % 97 + n)
    idx = make_index(x, w=w, leaf_size=tau, l_max=l_max)
    ids, d2, err, st = run_knn(idx, q, k, stats=True, err=True)
    check_knn(x, q, k, ids, d2)
    # every distance within its stated a-priori bound (about 1.2e-7 relative)
    check_err(x, q, ids, d2, err)
    st = {f: v.cpu().numpy() for f, v in st.items()}
    assert np.all(st["rounds"] >= 1)
    assert np.all(st["rows_refined"] >= k)
    # the deviation stage sees only LB_SAX survivors and passes only candidates
    assert np.all(st["candidates"] <= st["rows_sigma"])
    assert np.all(st["rows_sigma"] <= st["rows_filtered"])
    idx.close()


def test_large_magnitude_data_scales_exactly():
    # Series and queries times 1024 (exact in float32): iSAX words and LB_SAX
    # change (the breakpoints are for z-normalised data) but the search stays
    # exact, and every distance key scales by exactly 2^20, so the id lists
    # equal the unscaled run's.  Bounds and thresholds here exceed the fp16
    # range that the filter's survivor queue stores quarters in (its per-query
    # power-of-2 scale keeps them in range).
    x, q = workload(20_000, 256, coll=9, per_level=2, ood=1)
    idx = make_index(x, w=16, leaf_size=500, l_max=2)
    ids, d2 = run_knn(idx, q, 10)
    idx.close()
    xb, qb = x * np.float32(1024.0), q * np.float32(1024.0)
    idx = make_index(xb, w=16, leaf_size=500, l_max=2)
    ids_b, d2_b, st = run_knn(idx, qb, 10, stats=True)
    idx.close()
    check_knn(xb, qb, 10, ids_b, d2_b)
    assert np.array_equal(ids_b, ids)
    assert np.array_equal(d2_b, d2 * np.float32(2.0 ** 20))
    print(f"[large magnitude] candidates {st['candidates'].float().mean().item():.0f}, "
          f"deviation stage {st['rows_sigma'].float().mean().item():.0f}", flush=True)


def test_knn_k128_and_skip_sequential_path():
    x, q = workload(15_000, 256, coll=5)
    idx = make_index(x, w=16, leaf_size=400, eapca_th=1.1)   # every query skips LB_SAX
    ids, d2, st = run_knn(idx, q, 128, stats=True)
    check_knn(x, q, 128, ids, d2)
    assert np.all(st["path"].cpu().numpy() == 1)
    assert int(st["rows_sigma"].sum().item()) == 0
    idx.close()


def test_results_do_not_depend_on_access_path():
    x, q = workload(30_000, 256, coll=6, per_level=4)
    ref = None
    for tau, l_max, eth in ((10_000, 1, 0.0), (300, 0, 0.0), (1000, 4, 0.0), (2000, 1, 1.1), (1, 1, 0.0)):
        if tau == 1:
            x2, q2 = x[:3000], q
        else:
            x2, q2 = x, q
        idx = make_index(x2, w=16, leaf_size=tau, l_max=l_max, eapca_th=eth)
        ids, d2 = run_knn(idx, q2, 10)
        if tau == 1:
            check_knn(x2, q2, 10, ids, d2)
        elif ref is None:
            ref = (ids, d2)
            check_knn(x, q, 10, ids, d2)
        else:
            assert np.array_equal(ids, ref[0])
            assert np.array_equal(d2, ref[1])    # per-pair summation order is fixed
        idx.close()


def test_overflow_fallback_rounds():
    # One series per leaf and a seed that cannot fill k = 128: every series is
    # an LB_SAX survivor and the candidate list (a handful of entries per
    # filter wavefront) overflows, so the first round refines only about a
    # thousand candidates per query and its 128-th key is loose (about the
    # 12 % quantile of the distances).  In the fallback round every
    # single-series item is its own block, whose top list never fills k, so
    # the bound does not tighten inside the round: every series below that
    # key (about 12,000 of 100,000) is appended, more than the 4096-entry
    # result pool holds.  A third round follows, with the bound from the
    # entries that fit; the answer still matches the oracle.
    x, q = workload(100_000, 64, coll=13, per_level=1, ood=1)
    idx = make_index(x, w=8, leaf_size=1, l_max=1, cand_per_query=16)
    ids, d2, st = run_knn(idx, q, 128, stats=True)
    check_knn(x, q, 128, ids, d2)
    rounds = st["rounds"].cpu().numpy()
    print(f"[fallback] rounds {rounds.tolist()}", flush=True)
    assert np.all(rounds >= 2)
    assert rounds.max() >= 3
    idx.close()


def test_pool_overflow_round_takes_the_main_path():
    # No seed (l_max = 0) and k = 128: BSF_k is +inf while the first round
    # filters, so every series is a candidate, and every wavefront run appends
    # up to 128 entries: the 4096-entry result pools overflow.  The list has
    # room for every series (8N entries per query: a wavefront's private slice
    # holds a few hundred, the shared overflow slice the rest), so no
    # candidate is dropped and the second round runs the filter, list and
    # refine again with the merged bound: its LB_SAX survivors are counted on
    # top of the first round's N (the fused scan, which needs no list, counts
    # none), and the answer equals the oracle.
    N = 40_000
    x, q = workload(N, 128, coll=15, per_level=1, ood=2)
    idx = make_index(x, w=16, leaf_size=500, l_max=0, cand_per_query=8 * N)
    ids, d2, st = run_knn(idx, q, 128, stats=True)
    check_knn(x, q, 128, ids, d2)
    rounds = st["rounds"].cpu().numpy()
    cand = st["candidates"].cpu().numpy()
    print(f"[pool] rounds {rounds.tolist()} candidates {cand.tolist()}", flush=True)
    assert np.all(rounds >= 2)
    assert np.all(cand[rounds >= 2] > N)
    idx.close()


def test_many_exact_duplicates_at_the_kth_distance():
    # 9,000 exact copies of one series (more than the 4096-entry result pool):
    # a query equal to it, or near it, has all of them at one distance.  The
    # pool takes entries by result key (d, id), not by distance alone, so the
    # rounds end and the answer is the copies with the smallest ids.
    x = G.random_walks(30_000, 128, coll=31).copy()
    dup = np.arange(7, 30_000, 3)[:9000]
    x[dup] = x[5]
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([31, 2])))
    near = x[5].astype(np.float64) + 0.01 * g.standard_normal(128)
    near = ((near - near.mean()) / near.std()).astype(np.float32)
    q = np.stack([x[5], near, x[20_000]]).astype(np.float32)
    for cpq in (0, 16):
        idx = make_index(x, w=16, leaf_size=1000, l_max=1, cand_per_query=cpq)
        ids, d2, st = run_knn(idx, q, 10, stats=True)
        oids, od = check_knn(x, q, 10, ids, d2)
        assert np.array_equal(ids, oids)
        assert list(ids[0]) == [5] + list(dup[:9]) and np.all(d2[0] == 0)
        print(f"[duplicates] cand_per_query {cpq}: rounds {st['rounds'].cpu().numpy().tolist()}", flush=True)
        idx.close()


def _grid_offsets(rng, n, m, delta, lim):
    """m integer vectors c_j (|c| <= lim) whose sums of squares are
    T_j = T_0 (1 + j delta), each rounded up to the next integer that the
    two adjusted coordinates reach as a sum of two squares (a few units in
    about 1e9).  Returns (c [m, n], T [m])."""
    from math import isqrt
    base = rng.integers(-(lim // 2), lim // 2 + 1, n).astype(np.int64)
    base[:2] = 0
    S = int((base ** 2).sum())
    T0 = S + lim * lim // 4
    cs, Ts = [], []
    for j in range(m):
        R = round(T0 * (1.0 + j * delta)) - S
        assert 0 <= R <= lim * lim
        c = base.copy()
        while True:
            a = isqrt(R)
            while a >= 0 and 2 * a * a >= R:
                b2 = R - a * a
                b = isqrt(b2)
                if b * b == b2:
                    break
                a -= 1
            if a >= 0 and 2 * a * a >= R:
                c[0], c[1] = a, isqrt(R - a * a)
                break
            R += 1
        cs.append(c)
        Ts.append(S + R)
    return np.stack(cs), np.asarray(Ts, dtype=np.int64)


@pytest.mark.parametrize("n,w,l_max", [(256, 16, 0), (256, 16, 2), (1024, 32, 1)])
def test_planted_near_ties_outside_the_tie_band(n, w, l_max):
    # Around each query's k-th position, 2k planted series whose exact squared
    # distances T_j 2^-42 are spaced 1.2e-6, 2e-6 or 3e-6 relative apart, just
    # outside the 1e-6 tie band.  The query and the offsets lie on grids the
    # float32 format holds exactly (query multiples of 2^-12 below 4 in
    # magnitude, offsets c 2^-21 with integer c), so the FP64 distances are
    # exact: the id lists must equal the oracle's, each distance within its
    # stated bound.
    N, k = 20_000, 10
    x = G.random_walks(N, n, coll=200 + n).copy()
    qsrc, _, _ = G.workload(x, [1, 5, 10], 2, coll=200 + n)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([n, 3])))
    lim = 8191
    qs = []
    slots = rng.permutation(N)
    used = 0
    for i, delta in enumerate([1.2e-6, 2e-6, 3e-6, 1.2e-6, 2e-6, 3e-6]):
        qv = np.clip(np.round(qsrc[i].astype(np.float64) * 4096.0) / 4096.0, -3.9, 3.9).astype(np.float32)
        c, T = _grid_offsets(rng, n, 2 * k, delta, lim)
        assert np.all(np.diff(T) / T[:-1] > 1e-6)
        y = (qv[None, :].astype(np.float64) + c * 2.0 ** -21).astype(np.float32)
        assert np.array_equal(y.astype(np.float64) - qv.astype(np.float64), c * 2.0 ** -21)  # exact
        pos = slots[used:used + 2 * k]
        used += 2 * k
        x[pos] = y
        qs.append(qv)
    q = np.stack(qs)
    idx = make_index(x, w=w, leaf_size=500, l_max=l_max)
    ids, d2, err = run_knn(idx, q, k, err=True)
    oids, od = check_knn(x, q, k, ids, d2)
    for i in range(len(q)):
        gaps = np.diff(od[i]) / od[i, :-1]
        assert np.all(gaps > 1e-6), gaps  # the planted spacing survives in FP64
    assert np.array_equal(ids, oids)
    check_err(x, q, ids, d2, err)
    idx.close()


def test_candidate_list_fallback_matches_main_path():
    x, q = workload(30_000, 256, coll=14, per_level=3)
    a = make_index(x, w=16, leaf_size=1000)
    b = make_index(x, w=16, leaf_size=1000, cand_per_query=64)
    ia, da, sa = run_knn(a, q, 10, stats=True)
    ib, db, sb = run_knn(b, q, 10, stats=True)
    assert np.array_equal(ia, ib) and np.array_equal(da, db)
    assert sb["rounds"].cpu().numpy().max() >= 2
    check_knn(x, q, 10, ia, da)
    a.close()
    b.close()


def test_filter_windows_and_single_chunk_series():
    # thousands of small leaves and out-of-distribution queries: a workgroup
    # of the LB_SAX filter takes several 256-item windows, and 64-point series
    # are refined in one chunk each
    x = G.random_walks(200_000, 64, coll=21)
    q = G.ood_queries(64, 64, coll=21)
    idx = make_index(x, w=8, leaf_size=16)
    ids, d2, st = run_knn(idx, q, 10, stats=True)
    check_knn(x, q, 10, ids, d2)
    kept = st["leaves_kept"].cpu().numpy()
    assert kept.sum() > 256 * 1024  # more items than one window per workgroup of a full grid
    idx.close()


def test_batch_composition_does_not_change_results():
    x, q = workload(20_000, 256, coll=8, per_level=5)
    idx = make_index(x, w=16, leaf_size=500)
    ids, d2 = run_knn(idx, q, 10)
    for i in (0, 7, len(q) - 1):
        a, b = run_knn(idx, q[i:i + 1], 10)
        assert np.array_equal(a[0], ids[i]) and np.array_equal(b[0], d2[i])
    idx.close()


# ------------------------------------------------------------- edge cases

def test_planted_ties_and_exact_matches():
    x = G.random_walks(8000, 128, coll=9).copy()
    x[5000] = x[17]
    x[6001] = x[17]
    x[7999] = x[17]
    q = np.stack([x[17], x[4000], (x[100] + x[101]) / 2]).astype(np.float32)
    idx = make_index(x, w=16, leaf_size=250)
    ids, d2 = run_knn(idx, q, 4)
    assert list(ids[0][:4]) == [17, 5000, 6001, 7999] and np.all(d2[0] == 0)
    assert ids[1][0] == 4000 and d2[1][0] == 0
    check_knn(x, q, 4, ids, d2)
    idx.close()


def test_tiny_collections():
    x = G.random_walks(1, 64, coll=10)
    idx = make_index(x, w=16, leaf_size=10)
    ids, d2 = run_knn(idx, x + np.float32(0.5), 1)
    assert ids[0, 0] == 0 and abs(d2[0, 0] - 64 * 0.25) < 1e-5
    idx.close()
    x = G.random_walks(50, 64, coll=10)
    q = G.ood_queries(3, 64, coll=10)
    idx = make_index(x, w=8, leaf_size=7)
    ids, d2 = run_knn(idx, q, 50)                  # k = N: a full sort
    check_knn(x, q, 50, ids, d2)
    idx.close()


def test_errors():
    hs = hs_mod()
    x = G.random_walks(500, 64, coll=12)
    xt = torch.from_numpy(x).to(DEV)
    with pytest.raises(hs.HSError) as e:
        hs.Index(xt, hs.Params(w=7))
    assert e.value.code == hs.HS_EINVAL
    with pytest.raises(hs.HSError):
        hs.Index(xt, hs.Params(card_bits=4))
    bad = x.copy()
    bad[3, 5] = np.nan
    with pytest.raises(hs.HSError) as e:
        hs.Index(torch.from_numpy(bad).to(DEV), hs.Params(w=8, leaf_size=50))
    assert e.value.code == hs.HS_EINVAL
    idx = hs.Index(xt, hs.Params(w=8, leaf_size=50))
    qt = xt[:2].clone()
    for k in (0, hs.HS_KMAX + 1, 501):
        with pytest.raises(hs.HSError) as e:
            idx.knn(qt, k)
        assert e.value.code == hs.HS_EINVAL
    qn = qt.clone()
    qn[1, 0] = math.inf
    with pytest.raises(hs.HSError) as e:
        idx.knn(qn, 3)
    assert e.value.code == hs.HS_EINVAL
    ws, need = idx.workspace(2, 3)
    ids = torch.empty((2, 3), dtype=torch.int64, device=DEV)
    d2 = torch.empty((2, 3), dtype=torch.float32, device=DEV)
    with pytest.raises(hs.HSError) as e:
        hs.hs_knn_exact(idx.h, qt.data_ptr(), 2, 3, ws.data_ptr(), need - 1, ids.data_ptr(), d2.data_ptr(),
                        None, None, 0)
    assert e.value.code == hs.HS_ENOMEM
    with pytest.raises(hs.HSError) as e:
        hs.hs_knn_exact(idx.h, None, 2, 3, ws.data_ptr(), need, ids.data_ptr(), d2.data_ptr(), None, None, 0)
    assert e.value.code == hs.HS_EINVAL
    # at most 2^24 - 1 queries per call (rejected before any access to the arrays)
    with pytest.raises(hs.HSError) as e:
        hs.hs_knn_exact(idx.h, qt.data_ptr(), 1 << 24, 3, ws.data_ptr(), need, ids.data_ptr(), d2.data_ptr(),
                        None, None, 0)
    assert e.value.code == hs.HS_EINVAL
    # Q = 0 is a no-op
    hs.hs_knn_exact(idx.h, qt.data_ptr(), 0, 3, ws.data_ptr(), need, ids.data_ptr(), d2.data_ptr(), None, None,
                    0)
    # the index still answers correctly after the failed calls
    a, b = run_knn(idx, x[:2], 3)
    check_knn(x, x[:2], 3, a, b)
    idx.close()


def test_batch_union_counters():
    # Distinct units read by the filter and refine of one batch: each at most
    # the per-query totals, the envelopes at least any one query's (a query
    # tests a chunk envelope once), and the results unchanged by the marking
    # variants of the kernels.  The same batch twice over tests no further
    # envelope: the chunks tested follow from the leaves the seeds keep.
    hs = hs_mod()
    x, q = workload(30_000, 256, coll=17, per_level=4)
    idx = make_index(x, w=16, leaf_size=500, l_max=2)
    qt = torch.from_numpy(q).to(DEV)
    ref = idx.knn(qt, 10)
    out = {}

    def call(qq, key):
        out[key] = idx.knn(qq, 10, stats=True)

    raw, words, env = hs.union_counts(idx, lambda: call(qt, "a"))
    ids, d2, st = out["a"]
    torch.cuda.synchronize()
    assert torch.equal(ids, ref[0]) and torch.equal(d2, ref[1])
    st = {f: v.cpu().numpy() for f, v in st.items()}
    print(f"[union] raw {raw} words {words} env {env}; per query sums {st['chunks_read'].sum()} "
          f"{st['rows_filtered'].sum()} {st['chunks_tested'].sum()}", flush=True)
    nch = idx.info.row_stride // 64
    assert 0 < raw <= st["chunks_read"].sum() and raw <= x.shape[0] * nch
    assert 0 < words <= st["rows_filtered"].sum() and words <= x.shape[0]
    assert st["chunks_tested"].max() <= env <= st["chunks_tested"].sum() and env <= idx.info.n_chunks
    q2 = torch.cat([qt, qt]).contiguous()
    raw2, words2, env2 = hs.union_counts(idx, lambda: call(q2, "b"))
    assert env2 == env
    assert torch.equal(out["b"][0][:len(q)], ref[0])
    idx.close()


def test_lds_probe_rates():
    # Both patterns run their lookups without writing the sink; the
    # conflict-free pattern is not slower than random symbols.
    hs = hs_mod()
    sink = torch.zeros(1, dtype=torch.int32, device=DEV)
    free = hs.hs_lds_probe(0, 512, 2, sink.data_ptr(), 0)
    rand = hs.hs_lds_probe(1, 512, 2, sink.data_ptr(), 0)
    torch.cuda.synchronize()
    print(f"[lds probe] conflict-free {free / 1e12:.2f} T/s, random {rand / 1e12:.2f} T/s", flush=True)
    assert 1e11 < rand <= 1.05 * free < 1e14
    assert int(sink.item()) == 0


def test_read_probe_reads_without_writing():
    hs = hs_mod()
    buf = torch.arange(1 << 22, dtype=torch.int32, device=DEV)  # 16 MiB
    before = buf.clone()
    gbs = hs.read_probe_gbs(buf, passes=3)
    torch.cuda.synchronize()
    assert 10.0 < gbs < 20000.0
    assert torch.equal(buf, before)
