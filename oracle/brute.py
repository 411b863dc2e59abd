"""FP64 brute-force exact k-NN (oracle; test infrastructure only).

Follows the k-NN query definition of Hercules Sec. 2 (the k series of the
collection with the smallest distance to the query) under the squared
Euclidean distance used for whole matching (Sec. 2, UCR-Suite paragraph:
squared distances).  Ties are broken by the smaller row index; the result is
sorted by (distance, id) ascending.

``knn`` runs the C/OpenMP implementation in ``knn_brute.c`` (built by
``oracle/build.py``); ``knn_numpy`` is an independent numpy twin for tiny
inputs.  Both are plain definitions: no pruning, no early abandoning.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libknn_brute.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        lib.oracle_knn_brute.restype = ctypes.c_int
        lib.oracle_knn_brute.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32]
        lib.oracle_pair_dist.restype = ctypes.c_int
        lib.oracle_pair_dist.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        _LIB = lib
    return _LIB


def threads() -> int:
    """Threads the C oracle uses by default (OpenMP max threads)."""
    return int(_lib().oracle_threads())


def knn(x: np.ndarray, q: np.ndarray, k: int, threads: int = 0):
    """Exact k-NN of each row of ``q`` among the rows of ``x`` (float32 inputs).

    Returns (ids int64 [Q, k], d2 float64 [Q, k]) sorted by (d2, id).
    Raises ValueError on invalid arguments.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    if x.ndim != 2 or q.ndim != 2 or x.shape[1] != q.shape[1]:
        raise ValueError("x and q must be 2-D with equal row length")
    N, n = x.shape
    Q = q.shape[0]
    ids = np.empty((Q, k), dtype=np.int64)
    d2 = np.empty((Q, k), dtype=np.float64)
    rc = _lib().oracle_knn_brute(x.ctypes.data, N, n, q.ctypes.data, Q, k, ids.ctypes.data, d2.ctypes.data,
                                 int(threads))
    if rc != 0:
        raise ValueError(f"oracle_knn_brute failed ({rc})")
    return ids, d2


def knn_chunked(chunks, q: np.ndarray, k: int, threads: int = 0):
    """Exact k-NN over a collection given as consecutive row chunks (an
    iterable of float32 [rows, n] arrays, rows numbered from 0 across them):
    each chunk's own top-k by ``knn``, ids offset by the chunk's first row,
    merged with the running top-k by (d2, id).  The k nearest of the whole
    collection are among the union of the chunks' k nearest, so the merge is
    exact.  Returns (ids int64 [Q, k], d2 float64 [Q, k])."""
    q = np.ascontiguousarray(q, dtype=np.float32)
    Q = q.shape[0]
    best_i = np.empty((Q, 0), dtype=np.int64)
    best_d = np.empty((Q, 0), dtype=np.float64)
    base = 0
    for x in chunks:
        rows = x.shape[0]
        kk = min(k, rows)
        ci, cd = knn(x, q, kk, threads)
        ids = np.concatenate([best_i, ci + base], axis=1)
        ds = np.concatenate([best_d, cd], axis=1)
        keep = min(k, ids.shape[1])
        order = np.lexsort((ids, ds), axis=1)[:, :keep]   # primary key d2, then id
        best_i = np.take_along_axis(ids, order, axis=1)
        best_d = np.take_along_axis(ds, order, axis=1)
        base += rows
    if best_i.shape[1] < k:
        raise ValueError("k exceeds the collection")
    return best_i, best_d


def pair_dist(x: np.ndarray, q: np.ndarray, qidx, rows) -> np.ndarray:
    """FP64 squared distances d(q[qidx[p]], x[rows[p]]) for sampled pairs."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    qidx = np.ascontiguousarray(qidx, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if qidx.shape != rows.shape:
        raise ValueError("qidx and rows must have the same shape")
    out = np.empty(rows.shape, dtype=np.float64)
    rc = _lib().oracle_pair_dist(x.ctypes.data, x.shape[0], x.shape[1], q.ctypes.data, q.shape[0],
                                 qidx.ctypes.data, rows.ctypes.data, rows.size, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_pair_dist failed ({rc})")
    return out


def knn_numpy(x: np.ndarray, q: np.ndarray, k: int):
    """Numpy twin of ``knn`` for tiny inputs: full FP64 distance matrix."""
    x64 = np.asarray(x, dtype=np.float64)
    q64 = np.asarray(q, dtype=np.float64)
    if k < 1 or k > x64.shape[0]:
        raise ValueError("k out of range")
    ids = np.empty((q64.shape[0], k), dtype=np.int64)
    d2 = np.empty((q64.shape[0], k), dtype=np.float64)
    rowid = np.arange(x64.shape[0])
    for i, qq in enumerate(q64):
        diff = x64 - qq[None, :]
        d = np.einsum("ij,ij->i", diff, diff)
        order = np.lexsort((rowid, d))[:k]   # primary key d, then id
        ids[i] = order
        d2[i] = d[order]
    return ids, d2
