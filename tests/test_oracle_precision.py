"""Pins of the precision-form bound oracle (oracle/precision.py).

The bound is pinned by library routines (torch / numpy low-precision
conversions), by the triangle inequality it rests on (LB <= d64, checked on
random and on adversarial near-duplicate pairs), by its exact case (inputs
already representable: eps = 0 and LB = d64), and by float32-accumulated dot
products, whose worst-case error the accumulated form must absorb.
"""
import numpy as np
import pytest
import torch

from oracle import precision as P

pytestmark = pytest.mark.filterwarnings("ignore")


def _walks(rng, m, n):
    x = np.cumsum(rng.standard_normal((m, n)), axis=1)
    x = (x - x.mean(axis=1, keepdims=True)) / x.std(axis=1, keepdims=True)
    return x.astype(np.float32)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.standard_normal(100_000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 100_000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -2.5], np.float32)])
    v = v.astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(P.round_bf16(v), ref)


def test_bf16_ties_go_to_even():
    # 1 + 2^-8 lies half way between bf16 neighbours 1 and 1 + 2^-7: even is 1
    assert P.round_bf16(np.array([1.0 + 2.0 ** -8], np.float32))[0] == 1.0
    # 1 + 3 * 2^-8 lies half way between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert P.round_bf16(np.array([1.0 + 3 * 2.0 ** -8], np.float32))[0] == np.float32(1.0 + 2.0 ** -6)


def test_fp16_rounding_matches_numpy():
    rng = np.random.default_rng(2)
    v = (rng.standard_normal(10_000) * 3).astype(np.float32)
    np.testing.assert_array_equal(P.round_fp16(v), v.astype(np.float16).astype(np.float32))


@pytest.mark.parametrize("kind", [P.BF16, P.FP16])
def test_bound_never_exceeds_distance(kind):
    rng = np.random.default_rng(3 + kind)
    x = _walks(rng, 4000, 256)
    for i in range(5):
        q = x[rng.integers(0, len(x))] + rng.standard_normal(256).astype(np.float32) * 0.05 * (i + 1)
        q = ((q - q.mean()) / q.std()).astype(np.float32)
        d64 = np.sum((x.astype(np.float64) - q.astype(np.float64)) ** 2, axis=1)
        lb = P.lower_bound(q, x, kind)
        assert np.all(lb <= d64 * (1 + 1e-12) + 1e-12)
        # the bound is informative: tight for the nearest series
        j = int(np.argmin(d64))
        assert lb[j] > 0.5 * d64[j] or d64[j] < 1.0


@pytest.mark.parametrize("kind", [P.BF16, P.FP16])
def test_bound_on_near_duplicates(kind):
    # adversarial: series that differ from the query below the low-precision
    # resolution -- the bound must fall to (near) zero, never above d64
    rng = np.random.default_rng(5)
    q = _walks(rng, 1, 128)[0]
    x = q[None, :] + (rng.standard_normal((500, 128)) * 1e-4).astype(np.float32)
    x[0] = q
    d64 = np.sum((x.astype(np.float64) - q.astype(np.float64)) ** 2, axis=1)
    lb = P.lower_bound(q, x, kind)
    assert np.all(lb <= d64 + 1e-15)
    assert lb[0] == 0.0


@pytest.mark.parametrize("kind", [P.BF16, P.FP16])
def test_bound_is_exact_for_representable_inputs(kind):
    rng = np.random.default_rng(6)
    x = P.round_low((rng.standard_normal((200, 64)) * 2).astype(np.float32), kind)
    q = P.round_low((rng.standard_normal(64) * 2).astype(np.float32), kind)
    d64 = np.sum((x.astype(np.float64) - q.astype(np.float64)) ** 2, axis=1)
    np.testing.assert_allclose(P.lower_bound(q, x, kind), d64, rtol=1e-12)


def test_accumulation_factor_small_and_monotone():
    assert P.accumulation_factor(256) == pytest.approx(256 * 2.0 ** -23, rel=1e-4)
    assert P.accumulation_factor(1024) > P.accumulation_factor(256)


@pytest.mark.parametrize("kind", [P.BF16, P.FP16])
def test_accumulated_form_is_a_lower_bound(kind):
    # acc: the dot product accumulated in float32 in sequential order (one
    # rounding per addition, a worst-case-like order); the accumulated form
    # must stay below the exact low-precision bound's basis and below d64
    rng = np.random.default_rng(7)
    x = _walks(rng, 2000, 256)
    q = x[10] + rng.standard_normal(256).astype(np.float32) * 0.1
    q = ((q - q.mean()) / q.std()).astype(np.float32)
    ql = P.round_low(q, kind)
    xl = P.round_low(x, kind)
    acc = np.zeros(len(x), np.float32)
    for j in range(256):
        acc = (acc + (xl[:, j] * ql[j]).astype(np.float32)).astype(np.float32)
    d64 = np.sum((x.astype(np.float64) - q.astype(np.float64)) ** 2, axis=1)
    lb_acc = P.lower_bound_from_dot(q, x, kind, acc, 256)
    lb = P.lower_bound(q, x, kind)
    assert np.all(lb_acc <= d64 * (1 + 1e-12))
    assert np.all(lb_acc <= lb + 1e-9)
    # and it loses little: the accumulation slack is ~g (||q~||^2 + ||x~||^2)
    assert np.max(lb - lb_acc) < 0.1
