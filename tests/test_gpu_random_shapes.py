"""Seeded random shapes through both forms, against the FP64 oracle.

Each case draws a collection size, series length, word length w (dividing
n), leaf size, seed leaves, k, the query mix (noise levels and
out-of-dataset walks), and sometimes exact duplicates; the plain form must
match the oracle and the precision form (bf16 or fp16 copy) must return the
plain form's ids and distances.
"""
import numpy as np
import pytest
import torch

from paper_2212_13297_amd import datagen as G
from parity import check_knn

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def hs_mod():
    from paper_2212_13297_amd import hs
    hs.load()
    return hs


@pytest.mark.parametrize("seed", range(24))
def test_random_shape(seed):
    hs = hs_mod()
    rng = np.random.default_rng([2212, seed])
    n = int(rng.choice([64, 128, 192, 256, 320, 512, 1024]))
    w = int(rng.choice([w for w in (4, 5, 8, 10, 16, 20, 32, 40, 48, 64) if n % w == 0]))
    N = int(rng.integers(500, 30_000))
    tau = int(rng.choice([50, 200, 1000, 5000]))
    l_max = int(rng.integers(0, 6))
    k = min(int(rng.choice([1, 3, 10, 50, 100])), N)
    coll = 5000 + seed
    x = G.random_walks(N, n, coll=coll)
    q, _, _ = G.workload(x, [1, 5, 10], int(rng.integers(1, 4)), coll=coll)
    q = np.concatenate([q, G.ood_queries(int(rng.integers(0, 3)), n, coll=coll)])
    if seed % 5 == 0:
        x = x.copy()
        x[rng.integers(0, N, size=min(50, N))] = x[0]
    print(f"[case] seed={seed} N={N} n={n} w={w} tau={tau} l_max={l_max} k={k} Q={q.shape[0]}", flush=True)
    idx = hs.Index(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), hs.Params(w=w, leaf_size=tau, l_max=l_max))
    qt = torch.from_numpy(np.ascontiguousarray(q)).to(DEV)
    ids, d2 = idx.knn(qt, k)
    ids, d2 = ids.cpu().numpy(), d2.cpu().numpy()
    check_knn(x, q, k, ids, d2)
    idx.build_shadow(hs.HS_SHADOW_BF16 if seed % 2 == 0 else hs.HS_SHADOW_FP16)
    ids2, d22 = idx.knn_mixed(qt, k)[:2]
    torch.cuda.synchronize()
    assert np.array_equal(ids2.cpu().numpy(), ids)
    assert np.array_equal(d22.cpu().numpy(), d2)
    idx.close()
