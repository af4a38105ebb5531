"""Pins of the balanced-clustering oracle (Section 3.3; k-means, Section 2)
against things other than itself (CPU): a library's pairwise distances, an
independent mean, planted clusters, and the defining properties of the
balanced clustering."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import balance


def test_assignment_is_the_closest_centre():
    """argmin_j ||2^8 x - C_j||^2, first minimum, equals scipy's pairwise
    squared distances (exact in float64 at these magnitudes), ties
    included."""
    g = np.random.default_rng(1)
    X = g.integers(-127, 128, (700, 12)).astype(np.int8)
    C = g.integers(-127 * 256, 127 * 256, (40, 12))
    C[7] = C[3]  # a tie: the lower index wins
    D = cdist(X.astype(np.float64) * 256, C.astype(np.float64), "sqeuclidean")
    assert (balance.assign(X, C) == D.argmin(axis=1)).all()
    assert not (balance.assign(X, C) == 7).any()


def test_update_is_the_rounded_mean():
    g = np.random.default_rng(2)
    X = g.integers(-127, 128, (500, 5)).astype(np.int8)
    a = g.integers(0, 9, 500)
    a[a == 4] = 3  # cluster 4 empty: keeps its centre
    prev = g.integers(-9999, 9999, (9, 5))
    C = balance.update(X, a, prev)
    for j in range(9):
        mem = X[a == j].astype(np.float64)
        if len(mem) == 0:
            assert (C[j] == prev[j]).all()
            continue
        mean = mem.mean(axis=0) * 256
        assert (np.abs(C[j] - mean) <= 0.5).all()
        # half up exactly: recompute with Python fractions on one coordinate
        from fractions import Fraction
        s = int(X[a == j, 0].astype(np.int64).sum())
        assert C[j, 0] == math.floor(Fraction(256 * s, len(mem)) + Fraction(1, 2))


def test_kmeans_recovers_planted_clusters():
    """Well-separated planted clusters, started from one point of each: the
    planted partition in one round, and k = 1 gives the global mean."""
    g = np.random.default_rng(3)
    cen = np.array([[-100] * 6, [100] * 6, [0] * 6, [100, -100] * 3])
    lab = g.integers(0, 4, 800)
    X = (cen[lab] + g.integers(-4, 5, (800, 6))).astype(np.int8)
    init = np.array([np.nonzero(lab == c)[0][0] for c in range(4)])
    C, a = balance.kmeans(X, init, 10)
    assert (a == lab).all()
    C1, a1 = balance.kmeans(X, np.array([5]), 3)
    assert (a1 == 0).all()
    assert (np.abs(C1[0] - X.astype(np.float64).mean(axis=0) * 256) <= 0.5).all()


@pytest.mark.parametrize("m,alpha", [(60, 0.3), (25, 0.5), (200, 0.1)])
def test_balanced_clustering_properties(m, alpha):
    """Every cluster of every group has at most m points, the groups
    partition the points, each level leaves at most alpha of its points to
    the next, the chosen k is the smallest the search admits (k - 1 fails
    unless k is the lower bound (1 - alpha) n' / m), and there are at most
    log_{1/alpha} n + 1 groups (Section 3.3)."""
    g = np.random.default_rng(4)
    cen = g.integers(-110, 110, (40, 8))
    n = 2500
    # uneven cluster weights, as real data has
    w = g.dirichlet(np.full(40, 0.4))
    X = (cen[g.choice(40, n, p=w)] + g.integers(-9, 10, (n, 8))).astype(np.int8)
    perm = lambda level, k: np.random.default_rng(77 + level).permutation(k)
    groups = balance.balanced(X, m, alpha, 8, perm)
    ids = np.concatenate([gr.point_ids for gr in groups])
    assert sorted(ids.tolist()) == list(range(n))
    assert len(groups) <= math.log(n) / math.log(1 / alpha) + 1
    rem = np.arange(n)
    for level, gr in enumerate(groups):
        sizes = np.bincount(gr.cluster)
        last = level == len(groups) - 1
        assert sizes.max() <= m or last
        assert len(gr.centers) == len(sizes) and (sizes > 0).all()
        n1 = len(rem)
        assert n1 - len(gr.point_ids) <= alpha * n1
        lo = max(1, math.ceil((1 - alpha) * n1 / m))
        k = gr.k_searched
        if k > lo:
            p = perm(level, n1)
            _, a = balance.kmeans(X[rem], p[:k - 1], 8)
            s = np.bincount(a, minlength=k - 1)
            assert (s[a] > m).sum() > alpha * n1, level
        rem = np.setdiff1d(rem, gr.point_ids)
    assert len(rem) == 0
