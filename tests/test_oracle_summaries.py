"""Pins for the oracle's summaries and lower bounds (Hercules Sec. 2, Sec. 3.2).

Each function is tied to something other than its own formula: the normal CDF
computed independently with erfc, scipy's quantile function, closed forms of
simple series, exhaustive search on tiny inputs, the lower-bound invariant
(every bound <= the true squared distance, "no false dismissals", Sec. 2),
cases where a bound must be attained exactly, and the split example the paper
prints.
"""
import math
import os

import numpy as np
import pytest
from scipy.stats import norm

from oracle import summaries as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------- breakpoints

def test_breakpoints_are_normal_quantiles():
    b = S.breakpoints(256)
    assert b[0] == -math.inf and b[256] == math.inf
    for j in range(1, 256):
        phi = 0.5 * math.erfc(-b[j] / math.sqrt(2.0))   # independent CDF
        assert abs(phi - j / 256) < 1e-15
    np.testing.assert_allclose(b[1:-1], norm.ppf(np.arange(1, 256) / 256), rtol=0, atol=1e-13)
    assert b[128] == 0.0
    np.testing.assert_allclose(b[1:128], -b[255:128:-1], rtol=0, atol=1e-15)
    assert np.all(np.diff(b) > 0)


def test_breakpoints_card4_textbook():
    # quartiles of N(0, 1): +-0.6744897501960817 and 0
    b = S.breakpoints(4)
    np.testing.assert_allclose(b[1:4], [-0.6744897501960817, 0.0, 0.6744897501960817], atol=1e-15)


# --------------------------------------------------------------------- PAA

def test_paa_closed_forms():
    n, w = 256, 16
    ramp = np.arange(n, dtype=np.float64)
    l = n // w
    np.testing.assert_allclose(S.paa(ramp, w), np.arange(w) * l + (l - 1) / 2, rtol=0, atol=1e-12)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((10, n)).astype(np.float32)
    np.testing.assert_allclose((n / w) * S.paa(x, w).sum(1), x.astype(np.float64).sum(1), atol=1e-9)
    np.testing.assert_array_equal(S.paa(x, n), x.astype(np.float64))          # w = n: identity
    np.testing.assert_allclose(S.paa(x, 1)[:, 0], x.astype(np.float64).mean(1), atol=1e-15)
    with pytest.raises(ValueError):
        S.paa(x, 15)


# --------------------------------------------------------------- iSAX word

def test_sax_word_brute_force():
    b = S.breakpoints(256)
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.standard_normal(2000) * 1.5, b[1:-1], [-50.0, 50.0, 0.0]])
    s = S.sax_word(v, b)
    for val, sym in zip(v, s.astype(np.int64)):
        count = sum(1 for j in range(1, 256) if b[j] <= val)
        assert sym == count
        assert b[sym] <= val < b[sym + 1]
    # a value exactly on a breakpoint belongs to the upper region
    assert S.sax_word(np.array([b[100]]), b)[0] == 100


# ------------------------------------------------------------------ LB_SAX

def test_lb_sax_hand_example_card4():
    # n = 4, w = 2, alphabet 4.  Query PAA (1.0, -1.0); word (0, 3) covers
    # (-inf, -0.67449) and [0.67449, inf).  Each delta = 1 + 0.6744897501960817.
    b = S.breakpoints(4)
    delta = 1.0 + 0.6744897501960817
    got = S.lb_sax(np.array([1.0, -1.0]), np.array([0, 3]), b, 4)
    assert abs(got - (4 / 2) * 2 * delta * delta) < 1e-12
    # the word of the query's own PAA gives 0
    assert S.lb_sax(np.array([1.0, -1.0]), np.array([3, 0]), b, 4) == 0.0


def test_lb_sax_is_tight_minimum_over_regions():
    # For w = 2 the bound is (n/w) * min over the word's box of |paa_q - p|^2;
    # compare against an exhaustive grid over each (finite-clipped) region.
    b = S.breakpoints(256)
    n, w = 32, 2
    rng = np.random.default_rng(5)
    for _ in range(20):
        pq = rng.standard_normal(2) * 2
        word = rng.integers(0, 256, size=2)
        best = 0.0
        for i in range(2):
            lo = max(b[word[i]], -12.0)
            hi = min(b[word[i] + 1], 12.0)
            grid = np.linspace(lo, hi, 20001)
            best += np.min((grid - pq[i]) ** 2)
        got = S.lb_sax(pq, word, b, n)
        assert got <= (n / w) * best + 1e-12
        assert abs(got - (n / w) * best) <= (n / w) * 1e-6


def test_lb_sax_lower_bounds_distance():
    b = S.breakpoints(256)
    rng = np.random.default_rng(2)
    n, w = 128, 16
    x = np.cumsum(rng.standard_normal((400, n)), 1)
    x = (x - x.mean(1, keepdims=True)) / x.std(1, keepdims=True)
    q = x[:20] + rng.standard_normal((20, n)) * 0.3
    words = S.sax_word(S.paa(x, w), b)
    for qq in q:
        lb = S.lb_sax(S.paa(qq, w), words, b, n)
        d = ((x - qq) ** 2).sum(1)
        assert np.all(lb <= d + 1e-9)
        assert lb.max() > 0


# ------------------------------------------------------------------- EAPCA

def test_segment_stats_closed_forms():
    l = 16
    ramp = np.arange(l, dtype=np.float64)
    mu, sd = S.segment_stats(ramp, np.array([l]))
    assert abs(mu[0] - (l - 1) / 2) < 1e-12
    assert abs(sd[0] - math.sqrt((l * l - 1) / 12)) < 1e-12     # population std of 0..l-1
    alt = np.tile([2.5, -2.5], 8)
    mu, sd = S.segment_stats(alt, np.array([4, 16]))
    np.testing.assert_allclose(mu, [0, 0], atol=1e-15)
    np.testing.assert_allclose(sd, [2.5, 2.5], atol=1e-15)
    const = np.full(12, 3.25)
    mu, sd = S.segment_stats(const, np.array([5, 12]))
    np.testing.assert_allclose(mu, [3.25, 3.25])
    np.testing.assert_allclose(sd, [0, 0], atol=1e-15)


def test_synopsis_is_envelope():
    rng = np.random.default_rng(4)
    mu = rng.standard_normal((50, 6))
    sd = rng.random((50, 6))
    z = S.synopsis(mu, sd)
    np.testing.assert_array_equal(z[:, 0], mu.min(0))
    np.testing.assert_array_equal(z[:, 1], mu.max(0))
    np.testing.assert_array_equal(z[:, 2], sd.min(0))
    np.testing.assert_array_equal(z[:, 3], sd.max(0))


def _leaf_syn(x, ends):
    mu, sd = S.segment_stats(x, ends)
    return S.synopsis(mu, sd)


def test_lb_eapca_exact_cases():
    rng = np.random.default_rng(6)
    n = 64
    x = rng.standard_normal(n)
    q = rng.standard_normal(n)
    # unit segments on a one-series leaf: sigma = 0, mu = x_j, so lb^2 = d exactly
    ends = np.arange(1, n + 1)
    mq, sq = S.segment_stats(q, ends)
    lb = S.lb_eapca(mq, sq, _leaf_syn(x[None], ends), ends)
    assert abs(lb - ((q - x) ** 2).sum()) < 1e-9
    # segments of length 8; per segment the query is a shifted and positively
    # scaled copy of the series around its segment mean: q = mu + c + a (x - mu).
    # Then d = sum l [c^2 + (a-1)^2 sd^2] and the bound is attained exactly.
    ends = np.arange(8, n + 1, 8)
    starts = np.concatenate([[0], ends[:-1]])
    qq = np.empty(n)
    expect = 0.0
    for s0, e0 in zip(starts, ends):
        seg = x[s0:e0]
        mu = seg.mean()
        sdv = math.sqrt(((seg - mu) ** 2).mean())
        a = rng.uniform(0.2, 3.0)
        c = rng.uniform(-2, 2)
        qq[s0:e0] = mu + c + a * (seg - mu)
        expect += (e0 - s0) * (c * c + (a - 1) ** 2 * sdv * sdv)
    mq, sq = S.segment_stats(qq, ends)
    lb = S.lb_eapca(mq, sq, _leaf_syn(x[None], ends), ends)
    d = ((qq - x) ** 2).sum()
    assert abs(lb - expect) < 1e-9
    assert abs(lb - d) < 1e-9


def test_lb_eapca_single_segment_znorm_is_zero():
    rng = np.random.default_rng(8)
    x = np.cumsum(rng.standard_normal((30, 128)), 1)
    x = (x - x.mean(1, keepdims=True)) / x.std(1, keepdims=True)
    q = x[0] + rng.standard_normal(128)
    q = (q - q.mean()) / q.std()
    ends = np.array([128])
    mq, sq = S.segment_stats(q, ends)
    assert S.lb_eapca(mq, sq, _leaf_syn(x, ends), ends) < 1e-20


def test_lb_eapca_lower_bounds_members():
    rng = np.random.default_rng(9)
    n = 256
    x = np.cumsum(rng.standard_normal((300, n)), 1)
    x = (x - x.mean(1, keepdims=True)) / x.std(1, keepdims=True)
    ends = S.equal_segmentation(n, 16)
    groups = np.array_split(np.arange(300), 10)
    syns = np.stack([_leaf_syn(x[g], ends) for g in groups])
    for qq in x[:10] + rng.standard_normal((10, n)) * 0.4:
        mq, sq = S.segment_stats(qq, ends)
        lbs = S.lb_eapca(mq, sq, syns, ends)
        for g, lb in zip(groups, lbs):
            d = ((x[g] - qq) ** 2).sum(1)
            assert lb <= d.min() + 1e-9
        assert lbs.max() > 0


# ------------------------------------------------------------------ H-split

def test_hsplit_golden_example():
    rows = [l for l in open(os.path.join(GOLDEN, "hsplit_example.txt")) if not l.startswith("#")]
    mu_min, mu_max, thr = map(float, rows[0].split())
    assert abs(S.hsplit_threshold(mu_min, mu_max) - thr) < 1e-15
    v = np.array([-0.25, -0.0751, -0.075, -0.0749, 0.10])
    np.testing.assert_array_equal(S.hsplit_goes_left(v, mu_min, mu_max), [True, True, False, False, False])


def test_choose_split_prefers_widest_weighted_range():
    mu = np.array([[0.0, 0.0], [0.1, 2.0], [0.2, 1.0]])
    sd = np.array([[1.0, 1.0], [1.5, 1.0], [1.2, 1.0]])
    ends = np.array([2, 4])
    assert S.choose_split(mu, sd, ends) == (1, 0)
    # a constant node cannot be split
    assert S.choose_split(np.ones((4, 2)), np.ones((4, 2)), ends) is None
    # equal weighted ranges: lowest segment first, mean before std
    mu = np.array([[0.0, 0.0], [1.0, 1.0]])
    sd = np.array([[0.0, 0.0], [1.0, 1.0]])
    assert S.choose_split(mu, sd, ends) == (0, 0)


def test_build_leaves_partition():
    from paper_2212_13297_amd import datagen as G
    x = G.random_walks(5000, 128)
    leaves, ends = S.build_leaves(x, 16, 300)
    allids = np.concatenate(leaves)
    assert sorted(allids.tolist()) == list(range(5000))
    assert max(len(l) for l in leaves) <= 300
    mu, sd = S.segment_stats(x, ends)
    for l in leaves:
        assert np.all(np.diff(l) > 0)
        z = S.synopsis(mu[l], sd[l])
        assert np.all(mu[l] >= z[:, 0]) and np.all(mu[l] <= z[:, 1])


def test_build_tree_has_the_leaves_of_build_leaves():
    from paper_2212_13297_amd import datagen as G
    x = G.random_walks(3000, 64, coll=8)
    leaves, ends = S.build_leaves(x, 8, 100)
    nodes, ends2 = S.build_tree(x, 8, 100)
    np.testing.assert_array_equal(ends, ends2)
    tree_leaves = sorted((nd["leaf"], nd["ids"]) for nd in nodes if nd["children"] is None)
    assert [p for p, _ in tree_leaves] == list(range(len(leaves)))
    for (p, ids), ref in zip(tree_leaves, leaves):
        np.testing.assert_array_equal(ids, ref)
    # every internal node's series are its children's, split without loss
    for nd in nodes:
        if nd["children"] is not None:
            a, b = nd["children"]
            np.testing.assert_array_equal(np.sort(np.concatenate([nodes[a]["ids"], nodes[b]["ids"]])), nd["ids"])


# ------------------------------------------------------ deviation codes

def test_sigma_codes_contain_the_deviation():
    from paper_2212_13297_amd import datagen as G
    x = G.random_walks(3000, 128, coll=41)
    _, sd = S.segment_stats(x, S.equal_segmentation(128, 16))
    h = S.sigma_step(sd)
    c = S.sigma_codes(sd, h).astype(np.float64)
    assert np.all(c * h <= sd) and np.all(sd < (c + 1) * h)
    assert c.max() == 255 and h * 256 > sd.max()


@pytest.mark.parametrize("n,w", [(128, 16), (256, 16), (256, 32), (96, 8)])
def test_lb_sax_sigma_is_a_lower_bound_above_lb_sax(n, w):
    # against the exact squared distance of every pair (brute force), and
    # never below LB_SAX of the same pair
    from paper_2212_13297_amd import datagen as G
    x = G.random_walks(1500, n, coll=42)
    q, _, _ = G.workload(x, [1, 10], 3, coll=42)
    q = np.concatenate([q, G.ood_queries(3, n, coll=42)])
    beta = S.breakpoints(256)
    ends = S.equal_segmentation(n, w)
    words = S.sax_word(S.paa(x, w), beta)
    _, sd = S.segment_stats(x, ends)
    h = S.sigma_step(sd)
    codes = S.sigma_codes(sd, h)
    x64 = x.astype(np.float64)
    for qi in q.astype(np.float64):
        d = ((x64 - qi) ** 2).sum(1)
        pq = S.paa(qi, w)
        _, sq = S.segment_stats(qi, ends)
        lb = S.lb_sax_sigma(pq, sq, words, codes, beta, h, n)
        lbs = S.lb_sax(pq, words, beta, n)
        assert np.all(lb <= d * (1 + 1e-12))
        assert np.all(lb >= lbs)
        assert np.mean(lb > lbs) > 0.5  # the deviation term adds something for most series


def test_lb_sax_sigma_closed_forms():
    # a series against itself: its symbols and codes contain its own PAA and
    # deviations, so the bound is 0; a constant query (deviation 0 in every
    # segment) against a series whose codes are c_i: the deviation term is
    # (n/w) sum (c_i h)^2 on top of LB_SAX
    from paper_2212_13297_amd import datagen as G
    n, w = 128, 8
    x = G.random_walks(200, n, coll=43)
    beta = S.breakpoints(256)
    ends = S.equal_segmentation(n, w)
    words = S.sax_word(S.paa(x, w), beta)
    _, sd = S.segment_stats(x, ends)
    h = S.sigma_step(sd)
    codes = S.sigma_codes(sd, h)
    for i in range(0, 200, 37):
        xi = x[i].astype(np.float64)
        assert S.lb_sax_sigma(S.paa(xi, w), S.segment_stats(xi, ends)[1], words[i], codes[i], beta, h, n) == 0.0
    qc = np.zeros(n)
    lb = S.lb_sax_sigma(S.paa(qc, w), np.zeros(w), words, codes, beta, h, n)
    extra = (n / w) * ((codes.astype(np.float64) * h) ** 2).sum(1)
    np.testing.assert_allclose(lb, S.lb_sax(S.paa(qc, w), words, beta, n) + extra, rtol=1e-12, atol=0)
