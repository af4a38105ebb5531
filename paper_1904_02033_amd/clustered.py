"""Clustering-based sublinear form of the distance stage (Algorithm 4;
clustering protocol, steps 5 and 8).

The server keeps two resident databases: the cluster centres (packed and
randomly permuted, as step 4 shuffles them) and the points, packed cluster by
cluster followed by the stash (stash points permuted and chunk-aligned).  Per
query:

  phase 1  HE distances to every centre (a batched linear scan of the centre
           database);
  select   the client decrypts and the u closest clusters are chosen in the
           clear -- a stand-in for the garbled-circuit top-k and the DORAM
           retrieval of steps 5-6, which are out of scope;
  phase 2  HE distances to every chunk that holds a point of a selected
           cluster, plus every stash chunk: an uneven per-query chunk list
           served by one batched call (the scheduler packs the lists);
  finish   exact top-k over the selected clusters' points (Algorithm 1),
           approximate top-k over the stash (Algorithm 2), exact top-k of
           the 2k candidates (Algorithm 4's last step).

Each resident database has its own mask key, so one query id never draws
the same mask twice.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import native as nat
from . import stage, topk


@dataclasses.dataclass
class Layout:
    slot_point: np.ndarray       # [C N] int64 point index per slot, -1 padding
    cluster_start: np.ndarray    # [n_clusters] first slot of each cluster
    cluster_end: np.ndarray      # [n_clusters] one past the last slot
    stash_start: int             # first stash slot (chunk aligned)
    stash_end: int

    def chunks_of(self, clusters: Sequence[int], N: int) -> np.ndarray:
        """Sorted chunks that hold at least one slot of the given clusters."""
        out = set()
        for c in clusters:
            s, e = int(self.cluster_start[c]), int(self.cluster_end[c])
            if e > s:
                out.update(range(s // N, (e - 1) // N + 1))
        return np.array(sorted(out), dtype=np.int64)

    def stash_chunks(self, N: int) -> np.ndarray:
        return np.arange(self.stash_start // N, (self.stash_end + N - 1) // N,
                         dtype=np.int64)


def pack_clusters(cluster_sizes: np.ndarray, stash_size: int, N: int,
                  stash_perm: np.ndarray) -> Layout:
    """Points are stored clusters first (cluster c's points consecutive, in
    cluster order) then the stash; slots follow the same order, the stash
    starting on a chunk boundary in the server's random order."""
    sizes = np.asarray(cluster_sizes, dtype=np.int64)
    n_clustered = int(sizes.sum())
    start = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    end = start + sizes
    stash_start = (n_clustered + N - 1) // N * N
    total = stash_start + stash_size
    C = (total + N - 1) // N
    slot = np.full(C * N, -1, dtype=np.int64)
    slot[:n_clustered] = np.arange(n_clustered, dtype=np.int64)
    slot[stash_start:stash_start + stash_size] = n_clustered + np.asarray(stash_perm)
    return Layout(slot, start, end, stash_start, stash_start + stash_size)


class ClusteredServer:
    """Resident centre and point databases of one clustered index.

    resident (gathered=False): the points are one resident NTT-form database
    packed cluster by cluster, and phase 2 scans the chunks that hold each
    query's clusters (shared chunks carry other clusters' points too).
    gathered=True: the points stay on the device as they are; phase 2 packs
    each query's selected clusters into fresh chunks, encoded on the fly, and
    scans the stash (its own resident database) in the same call
    (sanns_distances_gathered with the stash as its tail)."""

    def __init__(self, ctx: stage.Context, points: np.ndarray, cluster_sizes: np.ndarray,
                 centers: np.ndarray, stash_size: int, center_perm: np.ndarray,
                 stash_perm: np.ndarray, key_points: bytes, key_centers: bytes,
                 gathered: bool = False):
        if key_points == key_centers:
            raise ValueError("the two resident databases need distinct mask keys")
        self.ctx = ctx
        N = ctx.N
        self.gathered = gathered
        self.n_clusters = len(cluster_sizes)
        self.layout = pack_clusters(cluster_sizes, stash_size, N, stash_perm)
        if gathered:
            dev = torch.device("cuda", ctx.device)
            self.pts_dev = torch.as_tensor(np.ascontiguousarray(points)).to(dev)
            st = self.layout.slot_point[self.layout.stash_start:]
            self.stash_slot = np.full((len(st) + N - 1) // N * N, -1, dtype=np.int64)
            self.stash_slot[:len(st)] = st
            self.sdb = stage.encode_db(ctx, points, self.stash_slot)
            self.db = None
        else:
            self.db = stage.encode_db(ctx, points, self.layout.slot_point)
        self.center_slot = stage.linear_slot_map(self.n_clusters, N, center_perm)
        self.cdb = stage.encode_db(ctx, centers, self.center_slot)
        self.key_points, self.key_centers = key_points, key_centers
        self.n_points = len(points)
        self.next_qid = 0

    def take_qids(self, Q: int) -> np.ndarray:
        """Q query ids never used before under this index's two mask keys."""
        out = np.arange(self.next_qid, self.next_qid + Q, dtype=np.uint64)
        self.next_qid += Q
        return out

    # ---------------------------------------------------------------- phase 1
    def center_distances(self, ct: torch.Tensor, qids: torch.Tensor,
                         mode: int = nat.SANNS_MODE_BATCHED, stream=None):
        """Shares of every query's distances to every centre."""
        D = stage.Distances(self.ctx, self.cdb, ct.shape[0], mode=mode)
        return D.run(ct, self.key_centers, qids, stream)

    # ---------------------------------------------------------------- phase 2
    def work_list(self, selected: Sequence[Sequence[int]]) -> np.ndarray:
        """(query, chunk) pairs: chunks of each query's selected clusters,
        then the stash chunks."""
        N = self.ctx.N
        stash = self.layout.stash_chunks(N)
        work = []
        for q, cl in enumerate(selected):
            ks = np.union1d(self.layout.chunks_of(cl, N), stash)
            work += [(q, int(k)) for k in ks]
        return np.array(work, dtype=np.uint32).reshape(-1, 2)

    def point_distances(self, ct: torch.Tensor, qids: torch.Tensor,
                        selected: Sequence[Sequence[int]],
                        mode: int = nat.SANNS_MODE_BATCHED, stream=None):
        work = self.work_list(selected)
        D = stage.Distances(self.ctx, self.db, ct.shape[0], work=work, mode=mode)
        out, share = D.run(ct, self.key_points, qids, stream)
        return out, share, work

    # ------------------------------------------------- phase 2, gathered form
    def gather_plan(self, selected: Sequence[Sequence[int]]):
        """Per query, the points of its selected clusters packed into fresh
        chunks: (slot map [M N] int64 with -1 padding, the query of each chunk
        [M] uint32)."""
        N = self.ctx.N
        lay = self.layout
        slots, rows = [], []
        for q, cl in enumerate(selected):
            idx = np.concatenate([np.arange(lay.cluster_start[c], lay.cluster_end[c])
                                  for c in cl]) if len(cl) else np.zeros(0, np.int64)
            m = max(1, (len(idx) + N - 1) // N)
            blk = np.full(m * N, -1, dtype=np.int64)
            blk[:len(idx)] = idx
            slots.append(blk)
            rows += [q] * m
        return np.concatenate(slots), np.array(rows, dtype=np.uint32)

    def gather_plan_device(self, selected: Sequence[Sequence[int]], stream=None):
        """gather_plan built on the device from the clusters' point ranges
        (only the R = sum of |selected| ranges cross from the host): (slot map,
        device int64 [M N]; chunk queries [M] uint32)."""
        N = self.ctx.N
        lay = self.layout
        starts, lens, offs, rows = [], [], [], []
        base = 0
        for q, cl in enumerate(selected):
            cl = np.asarray(cl, dtype=np.int64)
            st = lay.cluster_start[cl].astype(np.int64)
            ln = (lay.cluster_end[cl] - lay.cluster_start[cl]).astype(np.int64)
            starts.append(st)
            lens.append(ln)
            offs.append(base + np.concatenate([[0], np.cumsum(ln)[:-1]]).astype(np.int64))
            m = max(1, int((ln.sum() + N - 1) // N))
            rows += [q] * m
            base += m * N
        dev = torch.device("cuda", self.ctx.device)
        host = np.stack([np.concatenate(starts), np.concatenate(lens), np.concatenate(offs)])
        rng = torch.as_tensor(host).to(dev)
        slot = torch.empty(base, dtype=torch.int64, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream()
        nat.sanns_slot_ranges(rng[0].data_ptr(), rng[1].data_ptr(), rng[2].data_ptr(),
                              rng.shape[1], slot.data_ptr(), base, s.cuda_stream)
        self._ranges = rng  # held until the next plan: the fill may still be queued
        return slot, np.array(rows, dtype=np.uint32)

    def point_distances_gathered(self, ct: torch.Tensor, qids: torch.Tensor,
                                 selected: Sequence[Sequence[int]], stream=None):
        """Phase 2 in the gathered form, one call: ((ct_out, shares, slot
        map (device), chunk queries) of the selected clusters' fresh chunks,
        (ct_out, shares) of the stash for every query, rows q Cs + k)."""
        if not self.gathered:
            raise ValueError("the index was built without gathered=True")
        slot, rq = self.gather_plan_device(selected, stream)
        out, share = stage.gathered_distances(self.ctx, self.pts_dev, slot, rq, ct,
                                              self.key_points, qids, tail=self.sdb,
                                              stream=stream)
        M = len(rq)
        return (out[:M], share[:M], slot, rq), (out[M:], share[M:])

    def requested_pairs(self, selected: Sequence[Sequence[int]]) -> int:
        """Encrypted distances that phase 2 delivers for requested points."""
        sz = self.layout.cluster_end - self.layout.cluster_start
        stash = self.layout.stash_end - self.layout.stash_start
        return int(sum(int(sz[list(cl)].sum()) + stash for cl in selected))


# ---------------------------------------------------------------- client side

def select_clusters(center_dist: np.ndarray, center_slot: np.ndarray, u: int
                    ) -> np.ndarray:
    """The u closest clusters from one query's reconstructed centre distances
    ([C N] in slot order): Algorithm 1 over (distance, cluster id)."""
    real = center_slot >= 0
    _, ids = topk.naive_topk(center_dist[real], center_slot[real], u)
    return ids[ids >= 0]


class QueryDistances:
    """Reconstructed distances of one query from the phase-2 outputs: rows m
    of (client, server) shares whose work entry names this query."""

    def __init__(self, client: np.ndarray, server: np.ndarray, work: np.ndarray, q: int,
                 N: int, t: int):
        rows = np.nonzero(work[:, 0] == q)[0]
        self.row = np.full(int(work[:, 1].max()) + 1, -1, dtype=np.int64)
        self.row[work[rows, 1].astype(np.int64)] = rows
        self.client, self.server, self.N, self.t = client, server, N, t

    def __call__(self, slots: np.ndarray) -> np.ndarray:
        slots = np.asarray(slots, dtype=np.int64)
        rows = self.row[slots // self.N]
        if (rows < 0).any():
            raise KeyError("a requested slot lies in a chunk this query did not scan")
        off = slots % self.N
        return topk.reconstruct(self.client[rows, off], self.server[rows, off], self.t)


def finish_query(dist, layout: Layout, selected: Sequence[int], k: int, l_stash: int
                 ) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 4's selection from reconstructed distances: exact top-k over
    the selected clusters' points, approximate top-k over the stash, exact
    top-k of the 2k candidates.  dist(slots) returns the distances of the
    given slots.  Returns (values, point ids) of the final k."""
    parts = [np.arange(layout.cluster_start[c], layout.cluster_end[c]) for c in selected]
    cl_slots = np.concatenate(parts) if parts else np.zeros(0, np.int64)
    a_v, a_i = topk.naive_topk(dist(cl_slots), layout.slot_point[cl_slots], k)
    st_slots = np.arange(layout.stash_start, layout.stash_end)
    b_v, b_i = topk.approx_topk(dist(st_slots), layout.slot_point[st_slots], k, l_stash)
    return topk.naive_topk(np.concatenate([a_v, b_v]), np.concatenate([a_i, b_i]), k)
