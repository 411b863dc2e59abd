"""Oracle of the precision form's lower bound (test infrastructure only).

The precision form returns the same exact k-NN as the plain method; what it
adds is a per-series lower bound computed from low-precision copies of the
series and of the query.  This module states that bound in float64, from its
definition, for the tests:

  sqrt(d(q, x)) >= ||q~ - x~||_2 - ||q - q~||_2 - ||x - x~||_2      (triangle inequality)

so LB = max(0, ||q~ - x~|| - eps_q - eps_x)^2 <= d(q, x), where v~ is v
rounded to bf16 or fp16 (round to nearest even).  When the dot product
q~.x~ is accumulated in float32 over K terms, |acc - q~.x~| <= g ||q~|| ||x~||
with g = K u' / (1 - K u') (u' = 2^-23 covers any rounding of each addition;
the products of two bf16 or two fp16 values are exact in float32), and since
2 ||q~|| ||x~|| <= ||q~||^2 + ||x~||^2,

  ||q~ - x~||^2 >= (1 - g)(||q~||^2 + ||x~||^2) - 2 acc.

Pins (tests/test_oracle_precision.py): bf16 rounding equals torch's
conversion, fp16 rounding equals numpy's; LB <= d64 on random and adversarial
pairs; LB = d64 when q and x are exactly representable; the accumulated form
never exceeds the exact one for float32-accumulated dot products.
"""
from __future__ import annotations

import numpy as np

BF16, FP16 = 1, 2


def round_bf16(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bf16 (ties to even), returned as float32 values."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def round_fp16(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest fp16 (ties to even), returned as float32 values."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def round_low(x: np.ndarray, kind: int) -> np.ndarray:
    return round_bf16(x) if kind == BF16 else round_fp16(x)


def accumulation_factor(K: int) -> float:
    """g of the float32 accumulation bound for K additions (unit 2^-23)."""
    u2 = 2.0 ** -23
    return K * u2 / (1.0 - K * u2)


def lower_bound(q: np.ndarray, x: np.ndarray, kind: int) -> np.ndarray:
    """LB(q, x_i) for every row of x, float64, exact low-precision distance."""
    q64 = np.asarray(q, dtype=np.float64)
    x64 = np.asarray(x, dtype=np.float64)
    ql = round_low(q, kind).astype(np.float64)
    xl = round_low(x, kind).astype(np.float64)
    eps_q = np.sqrt(np.sum((q64 - ql) ** 2))
    eps_x = np.sqrt(np.sum((x64 - xl) ** 2, axis=1))
    dl = np.sqrt(np.sum((xl - ql[None, :]) ** 2, axis=1))
    return np.maximum(dl - eps_q - eps_x, 0.0) ** 2


def lower_bound_from_dot(q: np.ndarray, x: np.ndarray, kind: int, acc: np.ndarray, K: int) -> np.ndarray:
    """LB with ||q~ - x~||^2 replaced by its accumulated-dot lower bound
    (1 - g)(||q~||^2 + ||x~||^2) - 2 acc, acc the float32-accumulated q~.x~."""
    q64 = np.asarray(q, dtype=np.float64)
    x64 = np.asarray(x, dtype=np.float64)
    ql = round_low(q, kind).astype(np.float64)
    xl = round_low(x, kind).astype(np.float64)
    eps_q = np.sqrt(np.sum((q64 - ql) ** 2))
    eps_x = np.sqrt(np.sum((x64 - xl) ** 2, axis=1))
    g = accumulation_factor(K)
    d2lo = (1.0 - g) * (np.sum(ql * ql) + np.sum(xl * xl, axis=1)) - 2.0 * np.asarray(acc, dtype=np.float64)
    return np.maximum(np.sqrt(np.maximum(d2lo, 0.0)) - eps_q - eps_x, 0.0) ** 2
