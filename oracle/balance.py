"""Oracle of the balanced clustering -- TEST INFRASTRUCTURE.

Only tests and the benchmark's CPU leg use this module.  Plain definitions,
written from the paper:

  k-means (Lloyd's heuristic, the clustering subroutine of Section 2):
      alternate assigning every point to its closest centre and moving every
      centre to the mean of its points.  Points are integer vectors; centres
      live on a grid of 2^-8 (integers, 8 fractional bits), the mean rounded
      half up to that grid, so every step is exact integer arithmetic.  A
      point's closest centre minimises ||2^8 x - C||^2, ties to the lowest
      index; an empty cluster keeps its centre.  The initial centres are the
      points at the given indices (a seeded random choice, passed in).
      Iteration stops when no assignment changes or after `iters` rounds.
  balanced clustering (Section 3.3 "Balanced Clustering and Stash"):
      for the points still unclustered, find the smallest k whose k-means
      clustering leaves at most an alpha fraction of them in clusters of more
      than m points; the clusters of at most m points form the next group,
      the points of the larger clusters are clustered again, until every
      cluster has at most m points.  The last groups from T on form the
      stash, which is searched by a linear scan.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

FRAC = 8  # fractional bits of the centres


def assign(X: np.ndarray, C: np.ndarray, block: int = 256) -> np.ndarray:
    """Index of the closest centre of every point: argmin_j ||2^8 x - C_j||^2
    (first minimum).  X [n][d] integers, C [k][d] integers (2^-8 units)."""
    Xs = X.astype(np.int64) << FRAC
    C = C.astype(np.int64)
    out = np.empty(len(X), dtype=np.int64)
    for s in range(0, len(X), block):
        diff = Xs[s:s + block, None, :] - C[None, :, :]
        out[s:s + block] = (diff * diff).sum(axis=2).argmin(axis=1)
    return out


def update(X: np.ndarray, a: np.ndarray, C_prev: np.ndarray) -> np.ndarray:
    """Centre j = mean of its points on the 2^-8 grid, rounded half up
    (floor(2^8 S / cnt + 1/2)); an empty cluster keeps its centre."""
    C = C_prev.astype(np.int64).copy()
    for j in range(len(C)):
        members = X[a == j].astype(np.int64)
        cnt = len(members)
        if cnt:
            S = members.sum(axis=0)
            C[j] = ((S << (FRAC + 1)) + cnt) // (2 * cnt)
    return C


def kmeans(X: np.ndarray, init_idx: np.ndarray, iters: int):
    """(centres [k][d] on the 2^-8 grid, assignment [n]): the assignment of
    the last round and the centres of its clusters."""
    C = X[np.asarray(init_idx)].astype(np.int64) << FRAC
    prev = None
    for it in range(iters):
        a = assign(X, C)
        if prev is not None and (a == prev).all():
            return C, a
        C = update(X, a, C)
        prev = a
    return C, prev


@dataclasses.dataclass
class Group:
    point_ids: np.ndarray     # points of this group (indices into the input)
    cluster: np.ndarray       # their cluster, 0 .. k_i - 1 (clusters renumbered)
    centers: np.ndarray       # [k_i][d] on the 2^-8 grid
    k_searched: int           # the k of the k-means run the group came from


def balanced(X: np.ndarray, m: int, alpha: float, iters: int,
             perm: Callable[[int, int], np.ndarray]) -> List[Group]:
    """Groups of clusters of at most m points.  perm(level, n') is a random
    permutation of the n' points still unclustered at that level; a k-means
    run with k centres starts from its first k."""
    rem = np.arange(len(X))
    groups: List[Group] = []
    level = 0
    while len(rem):
        n1 = len(rem)
        Xr = X[rem]
        p = perm(level, n1)

        def run(k):
            C, a = kmeans(Xr, p[:k], iters)
            sizes = np.bincount(a, minlength=k)
            return C, a, sizes, int((sizes[a] > m).sum())

        # smallest k with at most alpha n1 points in clusters above m: at
        # least (1 - alpha) n1 / m clusters are needed; double from there,
        # then bisect (the criterion is taken as monotone in k)
        lo = max(1, math.ceil((1 - alpha) * n1 / m))
        k = lo
        res = run(k)
        while res[3] > alpha * n1 and k < n1:
            lo = k + 1
            k = min(n1, 2 * k)
            res = run(k)
        hi, best = k, res
        while lo < hi:
            mid = (lo + hi) // 2
            r = run(mid)
            if r[3] <= alpha * n1:
                hi, best = mid, r
            else:
                lo = mid + 1
        C, a, sizes, nbig = best
        small = sizes[a] <= m
        if not small.any():  # no cluster shrank to m: the rest is one last group
            small[:] = True
        keep = np.nonzero(np.bincount(a[small], minlength=hi))[0]
        renum = np.full(hi, -1, dtype=np.int64)
        renum[keep] = np.arange(len(keep))
        groups.append(Group(rem[small], renum[a[small]], C[keep], hi))
        rem = rem[~small]
        level += 1
    return groups
