"""Serial FP64 exact k-NN by filter-and-refine (oracle; test infrastructure only).

A self-check of the pruning rules of Hercules' exact search (Sec. 3.4), run
on the CPU over the oracle's own leaves (``summaries.build_leaves``).  What
makes the search exact is that every rule only discards work whose outcome
cannot enter the result:

* The result R holds the k best (d, id) pairs found so far, in (d, id)
  order; BSF_k is the distance of its k-th entry (+inf while R is short).
* A leaf is discarded when its LB_EAPCA (Sec. 2, the segment mean/std
  envelope bound) exceeds BSF_k, a series when its LB_SAX (the PAA of the
  query against the series' iSAX word) exceeds BSF_k, and a series'
  distance stops accumulating once the partial sum exceeds BSF_k.  Each is a
  lower bound of the series' true distance, and BSF_k only decreases, so a
  discarded series could never precede R's k-th entry.
* BSF_k starts from the leaves of smallest LB_EAPCA, at most L_max of them
  while their bound is within BSF_k, refined in full (the approximate
  search).
* How the surviving leaves are read is an access-path choice: when too few
  leaves were discarded (fraction below EAPCA_TH), or too few series would
  be by LB_SAX (fraction below SAX_TH), their series are refined without the
  LB_SAX test; otherwise only the LB_SAX survivors are, each bound tested
  again against the current BSF_k.

The same search also runs over the tree (``TreeIndex``, ``exact_knn_tree``):
the approximate search and the candidate-leaf step take nodes from one
priority queue ordered by LB_EAPCA, as Sec. 3.4 describes, with internal
synopses made from their children's.  On one segmentation a parent's box
contains its children's, so no node's bound exceeds a descendant's: leaves
leave the queue in increasing bound order, and the tree picks the same seed
and candidate leaves as sorting every leaf's own bound (ties broken by leaf
position; the queue orders nodes by their first leaf's position too).

Readings: the paper's tests are strict (LB < BSF_k, d < BSF_k), which can
drop a series tied with the k-th; here a bound discards only when strictly
greater, and a refined series enters R when its (d, id) precedes the k-th
entry.  Partial sums are checked after every 64 points, in point order.  The
result must equal brute force on every path.
"""
from __future__ import annotations

import math

import numpy as np

from . import summaries as S


class Results:
    """k best (d, id) pairs in ascending (d, id) order; BSF_k is the k-th distance."""

    def __init__(self, k: int):
        self.k = k
        self.d = [math.inf] * k
        self.id = [None] * k

    @property
    def bsf(self) -> float:
        return self.d[-1]

    def _before(self, d, i, j):
        """(d, i) precedes entry j (an empty entry is preceded by anything)."""
        if d != self.d[j]:
            return d < self.d[j]
        return self.id[j] is None or i < self.id[j]

    def offer(self, d: float, i: int) -> None:
        if not self._before(d, i, self.k - 1):
            return
        j = self.k - 1
        while j > 0 and self._before(d, i, j - 1):
            self.d[j], self.id[j] = self.d[j - 1], self.id[j - 1]
            j -= 1
        self.d[j], self.id[j] = d, i


def refine(q64: np.ndarray, x_row: np.ndarray, bsf: float) -> float:
    """Squared ED in FP64 with early abandoning (UCR-Suite style, Sec. 2): the
    full sum, or the first 64-point partial sum that exceeds bsf."""
    diff = q64 - x_row.astype(np.float64)
    running = np.cumsum(diff * diff)
    over = np.nonzero(running[63::64] > bsf)[0]
    if over.size:
        return float(running[63 + 64 * int(over[0])])
    return float(running[-1])


class LeafIndex:
    """Leaves, their synopses and the iSAX words of every series."""

    def __init__(self, x: np.ndarray, w: int, tau: int, card: int = 256):
        self.x = np.asarray(x, dtype=np.float32)
        self.n = self.x.shape[1]
        self.w = w
        self.beta = S.breakpoints(card)
        self.leaves, self.ends = S.build_leaves(self.x, w, tau)
        mu, sd = S.segment_stats(self.x, self.ends)
        self.syn = np.stack([S.synopsis(mu[ids], sd[ids]) for ids in self.leaves])
        self.words = S.sax_word(S.paa(self.x, w), self.beta)


def _refine_all(res: Results, q64, x, rows):
    for r in rows:
        res.offer(refine(q64, x[r], res.bsf), int(r))


def _finish(index, q64, res: Results, L: int, seeded: list, kept: list, eapca_th: float, sax_th: float,
            stats: dict | None):
    """The search after the seed: LB_SAX filter or skip-sequential reading of
    the kept leaves (in leaf order), then the result lists."""
    x, leaves = index.x, index.leaves
    mu_q, sd_q = S.segment_stats(q64, index.ends)
    lb_leaf = S.lb_eapca(mu_q, sd_q, index.syn, index.ends)
    leaf_pruned = 1.0 - len(kept) / L

    def read_whole_leaves():
        for leaf in kept:
            if lb_leaf[leaf] <= res.bsf:   # BSF_k may have tightened meanwhile
                _refine_all(res, q64, x, leaves[leaf])

    series_pruned = None
    if leaf_pruned < eapca_th:
        path = "skipseq_eapca"
        read_whole_leaves()
    else:
        paa_q = S.paa(q64, index.w)
        bsf0 = res.bsf
        rows = np.concatenate([leaves[leaf] for leaf in kept]) if kept else np.zeros(0, dtype=np.int64)
        lb_rows = S.lb_sax(paa_q, index.words[rows], index.beta, index.n) if len(rows) else np.zeros(0)
        survivors = [(int(r), float(b)) for r, b in zip(rows, lb_rows) if b <= bsf0]
        series_pruned = 1.0 - len(survivors) / x.shape[0]
        if series_pruned < sax_th:
            path = "skipseq_sax"
            read_whole_leaves()
        else:
            path = "sax"
            for r, b in survivors:
                if b <= res.bsf:
                    res.offer(refine(q64, x[r], res.bsf), r)

    if stats is not None:
        stats.update(dict(path=path, leaves=L, visited=len(seeded), lclist=len(kept),
                          eapca_pr=leaf_pruned, sax_pr=series_pruned, seeded=list(seeded), kept=list(kept)))
    ids = np.asarray([i if i is not None else -1 for i in res.id], dtype=np.int64)
    return ids, np.asarray(res.d, dtype=np.float64)


def exact_knn(index: LeafIndex, q: np.ndarray, k: int, l_max: int = 1,
              eapca_th: float = 0.25, sax_th: float = 0.50, stats: dict | None = None):
    """Exact k-NN of one query.  Returns (ids int64 [k], d2 float64 [k])."""
    if k < 1 or k > index.x.shape[0]:
        raise ValueError("k out of range")
    q64 = np.asarray(q, dtype=np.float64)
    x, leaves = index.x, index.leaves
    L = len(leaves)
    res = Results(k)
    mu_q, sd_q = S.segment_stats(q64, index.ends)
    lb_leaf = S.lb_eapca(mu_q, sd_q, index.syn, index.ends)
    by_bound = sorted(range(L), key=lambda i: (lb_leaf[i], i))

    # initial BSF_k: the most promising leaves, refined in full
    seeded = []
    for leaf in by_bound[:l_max]:
        if lb_leaf[leaf] > res.bsf:
            break
        _refine_all(res, q64, x, leaves[leaf])
        seeded.append(leaf)
    rest = by_bound[len(seeded):]

    # the leaves LB_EAPCA cannot discard at this BSF_k, in leaf order
    kept = sorted(leaf for leaf in rest if lb_leaf[leaf] <= res.bsf)
    return _finish(index, q64, res, L, seeded, kept, eapca_th, sax_th, stats)


class TreeIndex(LeafIndex):
    """LeafIndex plus the tree above its leaves: each node's synopsis (a
    leaf's over its series, an internal node's the union of its children's)
    and the position of the first leaf under it."""

    def __init__(self, x: np.ndarray, w: int, tau: int, card: int = 256):
        super().__init__(x, w, tau, card)
        self.nodes, _ = S.build_tree(self.x, w, tau)
        nn = len(self.nodes)
        self.node_syn = [None] * nn
        self.first_leaf = [0] * nn
        # children are appended after their parent: a reverse sweep is bottom-up
        for v in range(nn - 1, -1, -1):
            node = self.nodes[v]
            if node["children"] is None:
                self.node_syn[v] = self.syn[node["leaf"]]
                self.first_leaf[v] = node["leaf"]
            else:
                a, b = node["children"]
                self.node_syn[v] = S.union_synopsis(self.node_syn[a], self.node_syn[b])
                self.first_leaf[v] = min(self.first_leaf[a], self.first_leaf[b])


def exact_knn_tree(index: TreeIndex, q: np.ndarray, k: int, l_max: int = 1,
                   eapca_th: float = 0.25, sax_th: float = 0.50, stats: dict | None = None):
    """Exact k-NN of one query through the tree's priority queue: the
    approximate search pops nodes in increasing LB_EAPCA until l_max leaves
    are refined (a node whose bound exceeds BSF_k ends it), pushing the
    children of internal nodes whose bound does not exceed BSF_k; the
    candidate-leaf step resumes the same queue with BSF_k fixed and collects
    the leaves it pops, sorted by leaf position.  Returns (ids, d2)."""
    import heapq
    if k < 1 or k > index.x.shape[0]:
        raise ValueError("k out of range")
    q64 = np.asarray(q, dtype=np.float64)
    res = Results(k)
    mu_q, sd_q = S.segment_stats(q64, index.ends)

    def bound(v):
        return float(S.lb_eapca(mu_q, sd_q, index.node_syn[v], index.ends))

    pq = [(bound(0), index.first_leaf[0], 0)]

    def expand(v):
        for c in index.nodes[v]["children"]:
            b = bound(c)
            if b <= res.bsf:
                heapq.heappush(pq, (b, index.first_leaf[c], c))

    seeded = []
    while len(seeded) < l_max and pq:
        b, _, v = heapq.heappop(pq)
        if b > res.bsf:
            pq.clear()
            break
        node = index.nodes[v]
        if node["children"] is None:
            _refine_all(res, q64, index.x, index.leaves[node["leaf"]])
            seeded.append(node["leaf"])
        else:
            expand(v)
    kept = []
    while pq:
        b, _, v = heapq.heappop(pq)
        if b > res.bsf:
            break
        node = index.nodes[v]
        if node["children"] is None:
            kept.append(node["leaf"])
        else:
            expand(v)
    return _finish(index, q64, res, len(index.leaves), seeded, sorted(kept), eapca_th, sax_th, stats)
