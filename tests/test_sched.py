"""The serving loop's admission scheduler (host logic, hs_sched_* entry points).

Checks FIFO batch formation per collection, the slot limit (busy), the
per-k-bucket batch capacity that the HBM budget regions impose, the stream
busy/idle protocol, and -- in a randomized simulation -- that every admitted
request runs in exactly one batch, in submission order per collection, in a
batch that fits its region.
"""
import random

import pytest

from paper_2212_13297_amd import hs

HS_OK, HS_EBUSY = hs.HS_OK, hs.HS_EBUSY


@pytest.fixture
def lib():
    return hs.load()


def make(C, S, slots, max_q):
    return hs.hs_sched_create(C, S, slots, max_q)


def test_fifo_batch_takes_largest_k_bucket(lib):
    h = make(2, 2, 10, [[4] * 8, [2, 2, 2, 2, 1, 1, 0, 0]])
    assert hs.hs_sched_submit(h, 0, 5, 1) == HS_OK
    assert hs.hs_sched_submit(h, 0, 100, 2) == HS_OK
    assert hs.hs_sched_submit(h, 1, 3, 3) == HS_OK
    assert hs.hs_sched_next(h, 0, 0) == (2, 128, [1, 2])
    assert hs.hs_sched_next(h, 0, 1) is None          # nothing left for collection 0
    assert hs.hs_sched_next(h, 1, 0) == (1, 4, [3])
    assert hs.hs_sched_in_system(h) == 3
    hs.hs_sched_complete(h, 0, 0)
    assert hs.hs_sched_in_system(h) == 1
    hs.hs_sched_destroy(h)


def test_slots_limit_and_release(lib):
    h = make(1, 1, 3, [[8] * 8])
    assert [hs.hs_sched_submit(h, 0, 1, t) for t in range(4)] == [HS_OK, HS_OK, HS_OK, HS_EBUSY]
    assert hs.hs_sched_next(h, 0, 0) == (4, 1, [0, 1, 2])
    assert hs.hs_sched_submit(h, 0, 1, 9) == HS_EBUSY  # running requests still hold their slots
    hs.hs_sched_complete(h, 0, 0)
    assert hs.hs_sched_submit(h, 0, 1, 9) == HS_OK
    hs.hs_sched_destroy(h)


def test_cancel_withdraws_queued_requests_only(lib):
    h = make(2, 1, 4, [[4] * 8, [4] * 8])
    for t, c in ((10, 0), (11, 0), (12, 1), (13, 0)):
        assert hs.hs_sched_submit(h, c, 1, t) == HS_OK
    assert hs.hs_sched_submit(h, 0, 1, 14) == HS_EBUSY   # four slots, all taken
    hs.hs_sched_cancel(h, 11)                           # queued: withdrawn, its slot freed
    assert hs.hs_sched_in_system(h) == 3
    assert hs.hs_sched_submit(h, 0, 1, 14) == HS_OK
    assert hs.hs_sched_next(h, 0, 0) == (4, 1, [10, 13, 14])  # FIFO without the withdrawn one
    with pytest.raises(hs.HSError):
        hs.hs_sched_cancel(h, 13)                       # in a formed batch: no longer queued
    with pytest.raises(hs.HSError):
        hs.hs_sched_cancel(h, 99)                       # unknown tag
    hs.hs_sched_cancel(h, 12)                           # the other collection's queue
    assert hs.hs_sched_next(h, 1, 0) is None
    hs.hs_sched_complete(h, 0, 0)
    assert hs.hs_sched_in_system(h) == 0
    hs.hs_sched_destroy(h)


def test_capacity_depends_on_k_bucket(lib):
    # regions hold 8 queries at small k, 2 at k in (32, 64], none beyond
    h = make(1, 2, 100, [[8, 8, 8, 8, 8, 8, 2, 0]])
    for t in range(5):
        hs.hs_sched_submit(h, 0, 1, t)
    hs.hs_sched_submit(h, 0, 64, 5)
    hs.hs_sched_submit(h, 0, 33, 6)
    with pytest.raises(hs.HSError):
        hs.hs_sched_submit(h, 0, 65, 7)                  # bucket 7 holds nothing
    # the k=64 request would push the batch to bucket 6, capacity 2: it waits
    assert hs.hs_sched_next(h, 0, 0) == (8, 1, [0, 1, 2, 3, 4])
    assert hs.hs_sched_next(h, 0, 0) is None            # stream 0 busy
    assert hs.hs_sched_next(h, 0, 1) == (2, 64, [5, 6])
    hs.hs_sched_destroy(h)


def test_bad_arguments(lib):
    with pytest.raises(hs.HSError):
        make(1, 1, 4, [[3] * 8])                          # not a power of two
    h = make(1, 1, 4, [[4] * 8])
    with pytest.raises(hs.HSError):
        hs.hs_sched_submit(h, 1, 1, 0)                    # no such collection
    with pytest.raises(hs.HSError):
        hs.hs_sched_submit(h, 0, 0, 0)                    # k < 1
    with pytest.raises(hs.HSError):
        hs.hs_sched_next(h, 0, 0, max_tags=2)             # tag buffer below the largest batch
    hs.hs_sched_destroy(h)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_randomized_simulation(lib, seed):
    rng = random.Random(seed)
    C, S, slots = 3, 2, 40
    max_q = [[rng.choice([4, 8, 16])] * 5 + [rng.choice([1, 2, 4])] * 2 + [rng.choice([0, 1])] for _ in range(C)]
    h = make(C, S, slots, max_q)
    submitted = {c: [] for c in range(C)}
    ks = {}
    running = {}
    ran = {c: [] for c in range(C)}
    tag = 0
    in_sys = 0
    for _ in range(3000):
        op = rng.random()
        if op < 0.5:
            c = rng.randrange(C)
            k = rng.randint(1, 128)
            b = max(0, (k - 1).bit_length())
            if max_q[c][b] == 0:
                with pytest.raises(hs.HSError):
                    hs.hs_sched_submit(h, c, k, tag)
            else:
                rc = hs.hs_sched_submit(h, c, k, tag)
                assert rc == (HS_EBUSY if in_sys >= slots else HS_OK)
                if rc == HS_OK:
                    submitted[c].append(tag)
                    ks[tag] = k
                    in_sys += 1
            tag += 1
        elif op < 0.8:
            c, s = rng.randrange(C), rng.randrange(S)
            r = hs.hs_sched_next(h, c, s)
            if (c, s) in running:
                assert r is None
                continue
            if r is None:
                continue
            qp, kb, tags = r
            assert 1 <= len(tags) <= qp and qp & (qp - 1) == 0 and qp < 2 * len(tags)
            kmax = max(ks[t] for t in tags)
            assert kb >= kmax and kb < 2 * kmax
            b = kb.bit_length() - 1
            assert len(tags) <= max_q[c][b]
            running[(c, s)] = tags
            ran[c].extend(tags)
        else:
            if running:
                (c, s) = rng.choice(sorted(running))
                hs.hs_sched_complete(h, c, s)
                in_sys -= len(running.pop((c, s)))
        assert hs.hs_sched_in_system(h) == in_sys
    for c in range(C):
        # FIFO per collection, each request in at most one batch
        assert ran[c] == submitted[c][:len(ran[c])]
    hs.hs_sched_destroy(h)
