"""The package's cleartext top-k (used after reconstruction) against the
oracle's Algorithms 1 and 2, including ties and ragged bins (CPU)."""
import numpy as np
import pytest

import oracle
from paper_1904_02033_amd import topk


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("k", [1, 3, 10, 40])
def test_naive_topk_matches_oracle_with_ties(seed, k):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 300))
    vals = g.integers(0, max(2, n // 4), n)        # many ties
    ids = g.permutation(n) + 1000
    v, i = topk.naive_topk(vals, ids, k)
    ov, oi = oracle.naive_topk(vals.tolist(), ids.tolist(), k)
    m = min(k, n)
    assert v[:m].tolist() == ov[:m] and i[:m].tolist() == oi[:m]
    assert (i[m:] == -1).all()


@pytest.mark.parametrize("n,l,k", [(1000, 100, 10), (1003, 100, 10), (97, 10, 3),
                                   (64, 64, 5), (500, 7, 7)])
def test_approx_topk_matches_algorithm2(n, l, k):
    g = np.random.default_rng(n + l)
    vals = g.integers(0, 50, n)
    ids = np.arange(n)
    v, i = topk.approx_topk(vals, ids, k, l)
    ov, oi = oracle.approx_topk(vals, ids, k, l)
    assert v.tolist() == ov and i.tolist() == oi


def test_reconstruct_and_recall():
    t = 16957441
    d = np.array([0, 5, t - 1, 123456])
    r = np.array([7, t - 1, 3, 0])
    client = (d - r) % t
    assert (topk.reconstruct(client, r, t) == d).all()
    assert (topk.reconstruct(client, r, t, 2) == d >> 2).all()
    assert topk.recall(np.array([1, 2, 3]), np.array([3, 4, 1])) == pytest.approx(2 / 3)
    with pytest.raises(ValueError):
        topk.approx_topk(np.arange(10), np.arange(10), 5, 4)
