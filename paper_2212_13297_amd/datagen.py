"""Seeded synthetic inputs: random-walk collections and noisy query workloads.

This module holds the input recipe only (random numbers, cumulative sums and
z-normalisation of the inputs). None of the search method's arithmetic (PAA,
iSAX, EAPCA, distances, bounds) lives here, so both the HIP path and the CPU
oracle can take their inputs from it without sharing any of that arithmetic.

Recipe (Hercules, Sec. 4.1 "Datasets" and "Queries"):

* A series is a random walk: i.i.d. N(0, 1) steps, cumulatively summed, then
  z-normalised (population standard deviation) and cast to float32.  The
  float32 values are the canonical data.
* Rows are generated in chunks of 2**20 series.  Chunk ``c`` of collection
  ``coll`` draws from ``PCG64(SeedSequence([seed, coll, c]))``, so any chunk can
  be regenerated on its own and row ``i`` does not depend on how many rows are
  requested.
* A query of noise level ``p`` percent is a dataset row plus i.i.d.
  N(0, p/100) noise per point (the paper labels the noise *variance* as a
  percentage), re-z-normalised.  Source rows are drawn without replacement.
* Out-of-dataset ("ood") queries are fresh random walks from a seed disjoint
  from the collection's.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

CHUNK = 1 << 20
SEED_DATA = 20221
SEED_QUERY = 20222
SEED_NOISE = 20223
SEED_ARRIVAL = 20224


def _znorm_rows(a: np.ndarray) -> np.ndarray:
    """z-normalise each row of a float64 array in place (population std)."""
    a -= a.mean(axis=1, keepdims=True)
    sd = np.sqrt((a * a).mean(axis=1, keepdims=True))
    sd[sd < 1e-12] = 1.0
    a /= sd
    return a


def _walk_chunk(seed: int, coll: int, chunk: int, rows: int, n: int) -> np.ndarray:
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, coll, chunk])))
    steps = g.standard_normal((rows, n))
    np.cumsum(steps, axis=1, out=steps)
    return _znorm_rows(steps).astype(np.float32)


def _workers(workers):
    if workers is not None:
        return max(1, int(workers))
    return max(1, min(16, os.cpu_count() or 1))


def random_walks(N: int, n: int, seed: int = SEED_DATA, coll: int = 0,
                 workers: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Return ``N`` z-normalised random walks of length ``n`` as float32 [N, n].

    Chunks are generated in a thread pool (numpy releases the GIL inside its
    generators and ufuncs).  ``out`` may be a preallocated float32 [N, n]
    array, e.g. pinned host memory.
    """
    if N < 0 or n < 1:
        raise ValueError("N must be >= 0 and n >= 1")
    if out is None:
        out = np.empty((N, n), dtype=np.float32)
    elif out.shape != (N, n) or out.dtype != np.float32:
        raise ValueError("out must be float32 [N, n]")
    nchunks = (N + CHUNK - 1) // CHUNK

    def job(c):
        lo = c * CHUNK
        rows = min(CHUNK, N - lo)
        out[lo:lo + rows] = _walk_chunk(seed, coll, c, rows, n)

    if nchunks <= 1:
        for c in range(nchunks):
            job(c)
    else:
        with _cf.ThreadPoolExecutor(_workers(workers)) as ex:
            list(ex.map(job, range(nchunks)))
    return out


DEV_CHUNK = 1 << 18


def walk_chunk_device(chunk: int, rows: int, n: int, seed: int = SEED_DATA, coll: int = 0, device="cuda:0"):
    """Rows chunk * DEV_CHUNK .. + rows - 1 of a collection generated on the
    GPU (for collections too large for host memory): the same recipe -- i.i.d.
    N(0, 1) steps, cumulative sum, z-normalisation with the population std in
    FP64, cast to float32 -- drawn from torch's generator seeded per
    (seed, coll, chunk), so any chunk can be regenerated on its own.  A
    different stream of random numbers than ``random_walks``: a collection
    is generated one way or the other throughout."""
    import torch
    if rows < 1 or rows > DEV_CHUNK:
        raise ValueError("rows must be in [1, DEV_CHUNK]")
    g = torch.Generator(device=device)
    g.manual_seed(((seed * 1_000_003 + coll) * 1_000_003 + chunk) & ((1 << 63) - 1))
    x = torch.randn((rows, n), generator=g, dtype=torch.float64, device=device)
    torch.cumsum(x, dim=1, out=x)
    x -= x.mean(dim=1, keepdim=True)
    sd = torch.sqrt((x * x).mean(dim=1, keepdim=True))
    sd[sd < 1e-12] = 1.0
    x /= sd
    return x.to(torch.float32)


def walks_device(N: int, n: int, row0: int, rows: int, seed: int = SEED_DATA, coll: int = 0, device="cuda:0"):
    """Rows row0 .. row0 + rows - 1 (within one DEV_CHUNK chunk) of the
    N-row collection that ``walk_chunk_device`` generates."""
    c = row0 // DEV_CHUNK
    if (row0 + rows - 1) // DEV_CHUNK != c or row0 + rows > N:
        raise ValueError("rows must lie in one chunk of the collection")
    full = walk_chunk_device(c, min(DEV_CHUNK, N - c * DEV_CHUNK), n, seed, coll, device)
    off = row0 - c * DEV_CHUNK
    return full[off:off + rows].contiguous()


def query_sources(N: int, Q: int, seed: int = SEED_QUERY, coll: int = 0, tag: int = 0) -> np.ndarray:
    """Indices of ``Q`` distinct dataset rows used as query sources (int64)."""
    if Q > N:
        raise ValueError("cannot draw more distinct sources than rows")
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, coll, tag])))
    return g.choice(N, size=Q, replace=False).astype(np.int64)


def noisy_queries(sources: np.ndarray, noise_pct, seed: int = SEED_NOISE, coll: int = 0,
                  tag: int = 0) -> np.ndarray:
    """Perturb float32 source rows [Q, n] with N(0, p/100) noise, re-z-normalise.

    ``noise_pct`` is a scalar or a per-query array of percentages (variance
    labels: 5 means variance 0.05).
    """
    src = np.asarray(sources, dtype=np.float32)
    Q, n = src.shape
    var = np.broadcast_to(np.asarray(noise_pct, dtype=np.float64) / 100.0, (Q,))
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, coll, tag])))
    noise = g.standard_normal((Q, n)) * np.sqrt(var)[:, None]
    q = src.astype(np.float64) + noise
    return _znorm_rows(q).astype(np.float32)


def ood_queries(Q: int, n: int, coll: int = 0, tag: int = 0) -> np.ndarray:
    """Out-of-dataset queries: fresh random walks from a disjoint seed."""
    return random_walks(Q, n, seed=SEED_QUERY + 1000 + tag, coll=coll)


def workload(x: np.ndarray, noise_levels, per_level: int, coll: int = 0, tag: int = 0):
    """Queries built from rows of ``x``: ``per_level`` queries per noise level.

    Returns (queries float32 [L*per_level, n], source row ids int64, noise
    percentages float64), grouped by level in the order given.
    """
    levels = list(noise_levels)
    N = x.shape[0]
    src = query_sources(N, per_level * len(levels), coll=coll, tag=tag)
    pct = np.repeat(np.asarray(levels, dtype=np.float64), per_level)
    q = noisy_queries(x[src], pct, coll=coll, tag=tag)
    return q, src, pct


def poisson_arrivals(rate_qps: float, duration_s: float, seed: int = SEED_ARRIVAL, tag: int = 0) -> np.ndarray:
    """Arrival times (seconds, ascending) of a Poisson stream."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, tag])))
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate_qps)
        if t >= duration_s:
            break
        out.append(t)
    return np.asarray(out, dtype=np.float64)
