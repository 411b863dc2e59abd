"""FP64 summaries and lower bounds (oracle; test infrastructure only).

Written from Hercules (PVLDB 15(10), 2022):

* PAA and iSAX: Sec. 2, "Summarization Techniques" -- equal-length segments,
  each replaced by its mean (PAA); PAA values mapped to symbols of an alphabet
  (iSAX), 16 segments and an alphabet of 256 symbols.
* EAPCA: Sec. 2 -- each segment represented by its mean and standard
  deviation.
* Node synopsis: Sec. 3.2 (The Hercules Tree) -- per segment of the node's
  segmentation, the min/max over the node's series of the segment mean and of
  the segment standard deviation.
* H-split: Sec. 3.2 -- split on one segment's mean (or standard deviation) at
  the midpoint of its [min, max] range: values below the midpoint go left,
  values at or above it go right (the worked example splits at -0.075 for the
  range [-0.25, 0.10]).
* LB_SAX and LB_EAPCA: Sec. 2 names both lower-bounding distances but does not
  print their formulas; the readings used here are the standard ones and are
  derived in the docstrings below.
* Deviation codes (``sigma_codes``, ``lb_sax_sigma``): not in the paper; an
  8-bit code of each segment's standard deviation adds LB_EAPCA's deviation
  term to LB_SAX (derived below).

Readings where the paper is silent (each one listed in the design notes):

* Breakpoints are the equiprobable N(0, 1) quantiles Phi^-1(j / card),
  j = 1..card-1, with -inf / +inf at the two ends.
* A PAA value exactly on a breakpoint belongs to the upper region, so symbol
  s covers [beta_s, beta_{s+1}).
* w must divide n.
* Segment standard deviation is the population one (divide by the segment
  length).
* Split policy: the (segment, statistic) with the largest l_i * (max - min)^2,
  lowest segment first and mean before std on ties, skipping candidates that
  would leave a child empty.  Root segmentation: w equal segments.

All arithmetic is FP64 on the float32 inputs.
"""
from __future__ import annotations

import math
from statistics import NormalDist

import numpy as np


# --------------------------------------------------------------------- iSAX

def breakpoints(card: int = 256) -> np.ndarray:
    """Gaussian breakpoints beta_0..beta_card, beta_0 = -inf, beta_card = +inf.

    beta_j = Phi^-1(j / card) (equiprobable regions of N(0, 1)); the alphabet
    size 256 is Sec. 2's.  FP64 via the standard library's inverse normal CDF.
    """
    if card < 2:
        raise ValueError("card must be >= 2")
    nd = NormalDist()
    b = np.empty(card + 1, dtype=np.float64)
    b[0] = -math.inf
    b[card] = math.inf
    for j in range(1, card):
        b[j] = nd.inv_cdf(j / card)
    return b


def paa(x: np.ndarray, w: int) -> np.ndarray:
    """PAA over w equal segments (Sec. 2): the mean of each segment, FP64.

    x: [..., n] with w | n.  Returns [..., w].
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    if w < 1 or n % w:
        raise ValueError("w must divide n")
    return x.reshape(x.shape[:-1] + (w, n // w)).mean(axis=-1)


def sax_word(paa_vals: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """iSAX symbol per PAA value: s = #{j in 1..card-1 : beta_j <= paa}.

    The symbol's region is [beta_s, beta_{s+1}).  Returns uint8 for card 256.
    """
    inner = np.asarray(beta[1:-1], dtype=np.float64)
    s = np.searchsorted(inner, np.asarray(paa_vals, dtype=np.float64), side="right")
    return s.astype(np.uint8 if len(beta) - 1 <= 256 else np.int32)


def lb_sax(paa_q: np.ndarray, word: np.ndarray, beta: np.ndarray, n: int) -> np.ndarray:
    """Squared LB_SAX between the query's PAA and iSAX words (Sec. 2; the
    query side uses PAA(S_Q), not its word, as in the CSWorker step of
    Sec. 3.4).

    lb^2 = (n / w) * sum_i delta_i^2, delta_i the distance from paa_q[i] to the
    symbol's region [beta_s, beta_{s+1}].  Valid because, per segment,
    sum_seg (q - x)^2 >= (n/w) (paa_q - paa_x)^2 (Cauchy-Schwarz) and paa_x
    lies in the region.

    paa_q: [w]; word: [..., w] integer symbols.  Returns [...] FP64.
    """
    paa_q = np.asarray(paa_q, dtype=np.float64)
    word = np.asarray(word).astype(np.int64)
    w = paa_q.shape[-1]
    lo = beta[word]
    hi = beta[word + 1]
    below = np.where(paa_q < lo, lo - paa_q, 0.0)
    above = np.where(paa_q > hi, paa_q - hi, 0.0)
    delta = below + above
    return (n / w) * (delta * delta).sum(axis=-1)


# ------------------------------------------- deviation codes (an extension)
#
# Not in the paper: an 8-bit code per (series, segment) for the segment's
# standard deviation, which adds the deviation term of LB_EAPCA (Sec. 2) to
# LB_SAX.  Exactness does not depend on it; it only prunes more.

def sigma_step(sd: np.ndarray, levels: int = 256) -> float:
    """Code width h: the largest segment deviation spread over ``levels``
    codes, widened by 2^-20 so that every deviation lies below levels * h."""
    return float(np.max(sd)) * (1.0 + 2.0 ** -20) / levels if np.size(sd) else 1.0


def sigma_codes(sd: np.ndarray, h: float, levels: int = 256) -> np.ndarray:
    """Code of each segment deviation: c = floor(sd / h) (at most levels - 1),
    so that c h <= sd < (c + 1) h."""
    c = np.floor(np.asarray(sd, dtype=np.float64) / h).astype(np.int64)
    return np.clip(c, 0, levels - 1).astype(np.uint8 if levels <= 256 else np.int32)


def lb_sax_sigma(paa_q: np.ndarray, sd_q: np.ndarray, word: np.ndarray, code: np.ndarray, beta: np.ndarray,
                 h: float, n: int) -> np.ndarray:
    """Squared LB_SAX plus the deviation term:

        lb^2 = (n / w) * sum_i [delta_i^2 + gamma_i^2]

    delta_i as in ``lb_sax``; gamma_i the distance from the query's segment
    deviation sd_q[i] to the code's interval [c_i h, (c_i + 1) h].  Valid
    because, per segment of length l, sum (q - x)^2 = l [(mu_q - mu_x)^2 +
    (sd_q - sd_x)^2 + 2 sd_q sd_x (1 - rho)] >= l [(mu_q - mu_x)^2 +
    (sd_q - sd_x)^2] (rho <= 1, the inequality behind LB_EAPCA), with mu_x in
    the symbol's region and sd_x in the code's interval.

    paa_q, sd_q: [w]; word, code: [..., w] integers.  Returns [...] FP64.
    """
    paa_q = np.asarray(paa_q, dtype=np.float64)
    sd_q = np.asarray(sd_q, dtype=np.float64)
    w = paa_q.shape[-1]
    word = np.asarray(word).astype(np.int64)
    code = np.asarray(code).astype(np.float64)
    lo, hi = beta[word], beta[word + 1]
    delta = np.where(paa_q < lo, lo - paa_q, 0.0) + np.where(paa_q > hi, paa_q - hi, 0.0)
    slo, shi = code * h, (code + 1.0) * h
    gamma = np.where(sd_q < slo, slo - sd_q, 0.0) + np.where(sd_q > shi, sd_q - shi, 0.0)
    return (n / w) * (delta * delta + gamma * gamma).sum(axis=-1)


# -------------------------------------------------------------------- EAPCA

def equal_segmentation(n: int, m: int) -> np.ndarray:
    """Right endpoints r_1..r_m of m equal segments of [0, n) (r_m = n)."""
    if m < 1 or n % m:
        raise ValueError("m must divide n")
    return np.arange(1, m + 1, dtype=np.int64) * (n // m)


def segment_stats(x: np.ndarray, ends: np.ndarray):
    """EAPCA of each row over the segmentation with right endpoints ``ends``
    (Sec. 2 EAPCA; Sec. 3.2 segmentation SG = {r_1..r_m}, r_0 = 0).

    Segment i covers points [r_{i-1}, r_i).  mu = mean, sigma = population
    standard deviation.  x: [..., n].  Returns (mu, sigma), each [..., m].
    """
    x = np.asarray(x, dtype=np.float64)
    ends = np.asarray(ends, dtype=np.int64)
    starts = np.concatenate([[0], ends[:-1]])
    mus, sds = [], []
    for a, b in zip(starts, ends):
        seg = x[..., a:b]
        mu = seg.mean(axis=-1)
        dev = seg - mu[..., None]
        sd = np.sqrt((dev * dev).mean(axis=-1))
        mus.append(mu)
        sds.append(sd)
    return np.stack(mus, axis=-1), np.stack(sds, axis=-1)


def synopsis(mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    """Node synopsis z_i = (mu_min, mu_max, sd_min, sd_max) per segment over the
    node's series (Sec. 3.2).  mu, sd: [rows, m].  Returns [m, 4] FP64."""
    mu = np.asarray(mu, dtype=np.float64)
    sd = np.asarray(sd, dtype=np.float64)
    return np.stack([mu.min(0), mu.max(0), sd.min(0), sd.max(0)], axis=-1)


def _gap(v, lo, hi):
    """Distance from v to the closed interval [lo, hi]."""
    return np.maximum(0.0, np.maximum(lo - v, v - hi))


def lb_eapca(mu_q: np.ndarray, sd_q: np.ndarray, syn: np.ndarray, ends: np.ndarray) -> np.ndarray:
    """Squared LB_EAPCA between a query's EAPCA and a node synopsis.

    lb^2 = sum_i l_i [gap(mu_q,i, [mu_min, mu_max])^2 + gap(sd_q,i, [sd_min, sd_max])^2].
    Derivation (the paper cites the bound to DSTree without a formula): for one
    segment of length l, sum (q - x)^2 = l [(mu_q - mu_x)^2 + sd_q^2 + sd_x^2
    - 2 rho sd_q sd_x] >= l [(mu_q - mu_x)^2 + (sd_q - sd_x)^2] because the
    correlation rho <= 1; minimising over the synopsis box gives the bound.

    mu_q, sd_q: [m]; syn: [..., m, 4]; ends: [m].  Returns [...] FP64.
    """
    ends = np.asarray(ends, dtype=np.int64)
    lens = np.diff(np.concatenate([[0], ends])).astype(np.float64)
    syn = np.asarray(syn, dtype=np.float64)
    gm = _gap(np.asarray(mu_q, dtype=np.float64), syn[..., 0], syn[..., 1])
    gs = _gap(np.asarray(sd_q, dtype=np.float64), syn[..., 2], syn[..., 3])
    return (lens * (gm * gm + gs * gs)).sum(axis=-1)


# ------------------------------------------------------------------ H-split

def hsplit_threshold(vmin: float, vmax: float) -> float:
    """Midpoint of a segment statistic's [min, max] range (Sec. 3.2)."""
    return (vmin + vmax) / 2.0


def hsplit_goes_left(v, vmin: float, vmax: float):
    """Left child iff v lies in [min, (min+max)/2); right iff in [(min+max)/2, max]."""
    return np.asarray(v) < hsplit_threshold(vmin, vmax)


def choose_split(mu: np.ndarray, sd: np.ndarray, ends: np.ndarray):
    """Split policy reading: the candidate (segment i, statistic) with the
    largest l_i * (max - min)^2, lowest i first and mean before std on ties,
    whose midpoint split leaves both children non-empty.

    Returns (segment, stat) with stat 0 = mean, 1 = std, or None.
    """
    ends = np.asarray(ends, dtype=np.int64)
    lens = np.diff(np.concatenate([[0], ends])).astype(np.float64)
    cands = []
    for i in range(len(ends)):
        for st, v in ((0, mu[:, i]), (1, sd[:, i])):
            lo, hi = float(v.min()), float(v.max())
            cands.append((-(lens[i] * (hi - lo) ** 2), i, st))
    cands.sort()
    for negscore, i, st in cands:
        if negscore >= 0:
            break
        v = (mu if st == 0 else sd)[:, i]
        left = hsplit_goes_left(v, float(v.min()), float(v.max()))
        if left.any() and not left.all():
            return i, st
    return None


def build_leaves(x: np.ndarray, w: int, tau: int):
    """Leaf partition by repeated H-splits of every node holding more than
    ``tau`` series (Sec. 3.2 splitting, applied top-down to the whole batch).

    Returns (leaves, ends): ``leaves`` is a list of int64 arrays of row ids in
    in-order (left before right) leaf order, ids ascending inside each leaf;
    ``ends`` is the shared segmentation (w equal segments).
    """
    x = np.asarray(x)
    n = x.shape[1]
    ends = equal_segmentation(n, w)
    mu, sd = segment_stats(x, ends)
    leaves = []
    stack = [np.arange(x.shape[0], dtype=np.int64)]
    while stack:                      # depth-first, left child before right
        ids = stack.pop()
        if len(ids) <= tau:
            leaves.append(ids)
            continue
        pol = choose_split(mu[ids], sd[ids], ends)
        if pol is None:
            leaves.append(ids)
            continue
        i, st = pol
        v = (mu if st == 0 else sd)[ids, i]
        left = hsplit_goes_left(v, float(v.min()), float(v.max()))
        stack.append(ids[~left])
        stack.append(ids[left])
    return leaves, ends


def build_tree(x: np.ndarray, w: int, tau: int):
    """The H-split tree itself (Sec. 3.2-3.3): the same splits as
    ``build_leaves``, with the internal nodes kept.

    Returns (nodes, ends).  nodes[0] is the root; each node is a dict with
    ``ids`` (its series, ascending), ``children`` (indices of the left and
    right child, or None for a leaf) and ``leaf`` (the leaf's position in
    ``build_leaves``' in-order list, -1 for an internal node).
    """
    x = np.asarray(x)
    n = x.shape[1]
    ends = equal_segmentation(n, w)
    mu, sd = segment_stats(x, ends)
    nodes = [dict(ids=np.arange(x.shape[0], dtype=np.int64), children=None, leaf=-1)]
    stack = [0]
    n_leaves = 0
    while stack:                      # depth-first, left child before right
        v = stack.pop()
        ids = nodes[v]["ids"]
        pol = None if len(ids) <= tau else choose_split(mu[ids], sd[ids], ends)
        if pol is None:
            nodes[v]["leaf"] = n_leaves
            n_leaves += 1
            continue
        i, st = pol
        val = (mu if st == 0 else sd)[ids, i]
        left = hsplit_goes_left(val, float(val.min()), float(val.max()))
        nodes.append(dict(ids=ids[left], children=None, leaf=-1))
        nodes.append(dict(ids=ids[~left], children=None, leaf=-1))
        nodes[v]["children"] = (len(nodes) - 2, len(nodes) - 1)
        stack.append(len(nodes) - 1)
        stack.append(len(nodes) - 2)
    return nodes, ends


def union_synopsis(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """A parent's synopsis from its children's (Sec. 3.3, HSplitSynopsis): per
    segment the smallest minima and the largest maxima.  a, b: [m, 4]."""
    return np.stack([np.minimum(a[:, 0], b[:, 0]), np.maximum(a[:, 1], b[:, 1]),
                     np.minimum(a[:, 2], b[:, 2]), np.maximum(a[:, 3], b[:, 3])], axis=-1)
