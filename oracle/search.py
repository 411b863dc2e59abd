"""Serial FP64 run of Hercules' exact k-NN search (oracle; test infrastructure only).

Takes the steps of the paper's exact search (Sec. 3.4, the Exact-kNN
algorithm and its four steps) in order, over a flat list of leaves built by
``summaries.build_leaves``:

1. Approximate search (the Approx-kNN algorithm): leaves in ascending
   LB_EAPCA order; stop at the first whose bound exceeds BSF_k or after L_max
   leaves; refine every series of each visited leaf.
2. Candidate leaves (FindCandidateLeaves): the remaining leaves whose
   LB_EAPCA does not exceed BSF_k, kept in file (leaf) order; eapca_pr is the
   fraction pruned.
3. If eapca_pr < EAPCA_TH: skip-sequential scan of the candidate leaves.
   Otherwise candidate series (CSWorker): every series of a candidate leaf
   whose LB_SAX against PAA(query) does not exceed BSF_k; sax_pr is the
   fraction of all series pruned.
4. If sax_pr < SAX_TH: skip-sequential scan; otherwise refine the candidate
   series (CRWorker), re-checking each LB_SAX against the current BSF_k.

Readings (the paper's tests are strict ``<``, which can drop a candidate tied
with BSF_k): a node or series is pruned only when its bound is strictly
greater than BSF_k, and a refined series enters the result when (d, id)
precedes the current k-th entry lexicographically.  Results start as k
entries of (inf, none).  Refinement abandons a series once its partial sum
(FP64, points in order) exceeds BSF_k.  The thresholds choose an access path
only; all paths return the same result, which must equal brute force.
"""
from __future__ import annotations

import math

import numpy as np

from . import summaries as S


class Results:
    """k best (d, id) pairs in ascending order; BSF_k is the k-th distance."""

    def __init__(self, k: int):
        self.k = k
        self.d = [math.inf] * k
        self.id = [None] * k

    @property
    def bsf(self) -> float:
        return self.d[-1]

    def _precedes(self, d, i, j):
        if d != self.d[j]:
            return d < self.d[j]
        return self.id[j] is None or i < self.id[j]

    def offer(self, d: float, i: int) -> None:
        if not self._precedes(d, i, self.k - 1):
            return
        pos = self.k - 1
        while pos > 0 and self._precedes(d, i, pos - 1):
            self.d[pos] = self.d[pos - 1]
            self.id[pos] = self.id[pos - 1]
            pos -= 1
        self.d[pos] = d
        self.id[pos] = i


def refine(q64: np.ndarray, x_row: np.ndarray, bsf: float) -> float:
    """Squared ED in FP64 with early abandoning (UCR-Suite style, Sec. 2):
    returns the full sum, or a partial sum > bsf once it exceeds bsf."""
    diff = q64 - x_row.astype(np.float64)
    partial = np.cumsum(diff * diff)          # sequential running sums, FP64
    for end in range(63, len(partial), 64):   # checked after every 64 points
        if partial[end] > bsf:
            return float(partial[end])
    return float(partial[-1])


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


def exact_knn(index: LeafIndex, q: np.ndarray, k: int, l_max: int = 1,
              eapca_th: float = 0.25, sax_th: float = 0.50, stats: dict | None = None):
    """Exact k-NN of one query.  Returns (ids int64 [k], d2 float64 [k])."""
    if k < 1 or k > index.x.shape[0]:
        raise ValueError("k out of range")
    q64 = np.asarray(q, dtype=np.float64)
    x = index.x
    res = Results(k)

    mu_q, sd_q = S.segment_stats(q64, index.ends)
    lb_leaf = S.lb_eapca(mu_q, sd_q, index.syn, index.ends)
    L = len(index.leaves)
    order = sorted(range(L), key=lambda i: (lb_leaf[i], i))

    # Step 1: approximate search over at most l_max leaves
    visited = set()
    pos = 0
    while len(visited) < l_max and pos < L:
        leaf = order[pos]
        if lb_leaf[leaf] > res.bsf:
            break
        for r in index.leaves[leaf]:
            d = refine(q64, x[r], res.bsf)
            res.offer(d, int(r))
        visited.add(leaf)
        pos += 1

    # Step 2: candidate leaves, file order
    bsf = res.bsf
    lclist = sorted(i for i in order[pos:] if lb_leaf[i] <= bsf)
    eapca_pr = 1.0 - len(lclist) / L
    path = "sax"

    def skip_sequential():
        for leaf in lclist:
            if lb_leaf[leaf] > res.bsf:
                continue
            for r in index.leaves[leaf]:
                d = refine(q64, x[r], res.bsf)
                res.offer(d, int(r))

    sax_pr = None
    if eapca_pr < eapca_th:
        path = "skipseq_eapca"
        skip_sequential()
    else:
        # Step 3: candidate series by LB_SAX against PAA(query)
        paa_q = S.paa(q64, index.w)
        sclist = []
        for leaf in lclist:
            ids = index.leaves[leaf]
            lbs = S.lb_sax(paa_q, index.words[ids], index.beta, index.n)
            for r, lb in zip(ids, lbs):
                if lb <= bsf:
                    sclist.append((int(r), float(lb)))
        sax_pr = 1.0 - len(sclist) / x.shape[0]
        if sax_pr < sax_th:
            path = "skipseq_sax"
            skip_sequential()
        else:
            # Step 4: refine candidate series against the current BSF_k
            for r, lb in sclist:
                if lb > res.bsf:
                    continue
                d = refine(q64, x[r], res.bsf)
                res.offer(d, r)

    if stats is not None:
        stats.update(dict(path=path, leaves=L, visited=len(visited), lclist=len(lclist),
                          eapca_pr=eapca_pr, sax_pr=sax_pr))
    ids = np.asarray([i if i is not None else -1 for i in res.id], dtype=np.int64)
    return ids, np.asarray(res.d, dtype=np.float64)
