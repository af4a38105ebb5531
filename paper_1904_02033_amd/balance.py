"""Balanced clustering with a stash (Section 3.3 "Balanced Clustering and
Stash"), the server's preprocessing step before the clustering-based form.

The paper runs it with PyTorch k-means on GPUs (Section 5 "Environment"); here
the k-means rounds are the library's integer kernels (sanns_kmeans_*: exact
assignment to the closest centre on a 2^-8 grid, exact rounded means), and
this module holds only the search over k and the bookkeeping:

  for the points still unclustered, find the smallest k whose k-means
  clustering leaves at most an alpha fraction of them in clusters of more
  than m points (from the lower bound (1 - alpha) n' / m, doubling, then
  bisecting: the criterion is taken as monotone in k); the clusters of at
  most m points form the next group and the points of the larger ones are
  clustered again, until no point is left.  Groups from T on form the stash.

Random choices (the initial centres) are inputs: perm(level, n') returns a
random permutation of the n' points of a level, and a k-means run with k
centres starts from its first k.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np
import torch

from . import native as nat


class KMeans:
    """Device buffers of k-means rounds over one set of int8 points."""

    def __init__(self, points: torch.Tensor, stream=None):
        if points.dtype != torch.int8 or points.dim() != 2 or not points.is_cuda:
            raise ValueError("points must be a device int8 [n][d] tensor")
        self.X = points.contiguous()
        self.n, self.d = self.X.shape
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        dev = self.X.device
        self.flag = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws = None

    def _ws(self, k: int) -> torch.Tensor:
        nb = nat.sanns_kmeans_workspace(k, self.d)
        if self.ws is None or self.ws.numel() < nb:
            self.ws = torch.empty(nb, dtype=torch.uint8, device=self.X.device)
        return self.ws

    def run(self, init_idx: np.ndarray, iters: int):
        """(centres [k][d] int32 on the 2^-8 grid, assignment [n] int32, rounds
        run): the assignment of the last round and the centres of its
        clusters (an empty cluster keeps its centre)."""
        k = len(init_idx)
        dev = self.X.device
        s = self.stream.cuda_stream
        idx = torch.as_tensor(np.ascontiguousarray(init_idx, dtype=np.int64)).to(dev)
        C = torch.empty((k, self.d), dtype=torch.int32, device=dev)
        self.flag.zero_()
        nat.sanns_kmeans_init(self.X.data_ptr(), self.n, self.d, idx.data_ptr(), k,
                              C.data_ptr(), self.flag.data_ptr(), s)
        ws = self._ws(k)
        a = [torch.empty(self.n, dtype=torch.int32, device=dev) for _ in range(2)]
        prev = None
        for it in range(iters):
            cur = a[it % 2]
            self.flag.zero_()
            nat.sanns_kmeans_assign(self.X.data_ptr(), self.n, self.d, C.data_ptr(), k,
                                    0 if prev is None else prev.data_ptr(), cur.data_ptr(),
                                    self.flag.data_ptr(), ws.data_ptr(), ws.numel(), s)
            if prev is not None and int(self.flag.item()) == 0:
                return C, cur, it + 1
            nat.sanns_kmeans_update(self.X.data_ptr(), self.n, self.d, cur.data_ptr(), k,
                                    C.data_ptr(), 0, ws.data_ptr(), ws.numel(), s)
            prev = cur
        return C, prev, iters


@dataclasses.dataclass
class Group:
    point_ids: np.ndarray     # points of this group (indices into the input)
    cluster: np.ndarray       # their cluster, 0 .. k_i - 1
    centers: np.ndarray       # [k_i][d] int32 on the 2^-8 grid
    k_searched: int           # the k of the k-means run the group came from


@dataclasses.dataclass
class Balanced:
    groups: List[Group]
    kmeans_runs: int
    kmeans_rounds: int

    def stash(self, T: int) -> np.ndarray:
        """Points of the groups from T on (the stash, scanned linearly)."""
        parts = [g.point_ids for g in self.groups[T:]]
        return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)

    def index(self, T: int):
        """(cluster sizes, point order (clusters contiguous, groups < T), int8
        centres (rounded to the integer grid), group of each cluster, stash
        points): the inputs of the clustered form."""
        sizes, order, cents, grp = [], [], [], []
        for gi, g in enumerate(self.groups[:T]):
            o = np.argsort(g.cluster, kind="stable")
            order.append(g.point_ids[o])
            sizes.append(np.bincount(g.cluster, minlength=len(g.centers)))
            c = np.floor_divide(g.centers.astype(np.int64) + 128, 256)
            cents.append(np.clip(c, -127, 127).astype(np.int8))
            grp.append(np.full(len(g.centers), gi, dtype=np.int64))
        return (np.concatenate(sizes), np.concatenate(order), np.concatenate(cents),
                np.concatenate(grp), self.stash(T))


def balanced_clustering(points: np.ndarray, m: int, alpha: float, iters: int,
                        perm: Callable[[int, int], np.ndarray], device: int = 0) -> Balanced:
    """Groups of clusters of at most m points (the last group takes what is
    left if no cluster of a level shrinks to m points)."""
    if not 0 < alpha < 1 or m < 1:
        raise ValueError("need 0 < alpha < 1 and m >= 1")
    dev = torch.device("cuda", device)
    X = np.ascontiguousarray(points, dtype=np.int8)
    rem = np.arange(len(X))
    groups: List[Group] = []
    runs = rounds = 0
    level = 0
    while len(rem):
        n1 = len(rem)
        km = KMeans(torch.as_tensor(X[rem]).to(dev))
        p = perm(level, n1)

        def run(k):
            nonlocal runs, rounds
            C, a, r = km.run(p[:k], iters)
            runs += 1
            rounds += r
            a = a.cpu().numpy().astype(np.int64)
            sizes = np.bincount(a, minlength=k)
            return C.cpu().numpy(), a, sizes, int((sizes[a] > m).sum())

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
        C, a, sizes, _ = best
        small = sizes[a] <= m
        if not small.any():
            small[:] = True
        keep = np.nonzero(np.bincount(a[small], minlength=hi))[0]
        renum = np.full(hi, -1, dtype=np.int64)
        renum[keep] = np.arange(len(keep))
        groups.append(Group(rem[small], renum[a[small]], C[keep], hi))
        rem = rem[~small]
        level += 1
    return Balanced(groups, runs, rounds)
