"""Seeded problems for the parity tests: the same inputs (from synthdata) go
to the HIP path and to the oracle; nothing the HIP path computes is fed to
the oracle."""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

import oracle
import synthdata


@dataclasses.dataclass
class Problem:
    P: oracle.Params
    pts: np.ndarray          # [n][d] uint8 / int8
    queries: np.ndarray      # [Q][d] same dtype
    sk: np.ndarray           # [N] int8
    a: np.ndarray            # [Q][d][L][N] uint64
    e: np.ndarray            # [Q][d][N] int16
    slot: np.ndarray         # [C N] int64
    key: bytes
    qids: np.ndarray         # [Q] uint64

    @property
    def N(self):
        return self.P.N

    @property
    def C(self):
        return len(self.slot) // self.P.N

    @property
    def Q(self):
        return self.queries.shape[0]

    def qnorm2(self) -> np.ndarray:
        q = self.queries.astype(np.int64)
        return ((q * q).sum(axis=1) % self.P.t).astype(np.uint32)


def make_problem(N: int, L: int, t_bits: int, n: int, d: int, Q: int, dtype: str = "u8",
                 seed: int = 0, points: Optional[np.ndarray] = None,
                 queries: Optional[np.ndarray] = None, t: Optional[int] = None,
                 qs: Optional[Sequence[int]] = None) -> Problem:
    """t: the plain modulus (default: the prime of t_bits bits that the
    workloads use); qs: the RNS primes (default: the L largest NTT-friendly
    primes below 2^54)."""
    P = oracle.Params(N, list(qs) if qs is not None else oracle.rns_primes(N, L),
                      t if t is not None else oracle.plain_modulus(N, t_bits))
    g = np.random.default_rng(seed)
    if points is None:
        if dtype == "u8":
            points = g.integers(0, 256, (n, d)).astype(np.uint8)
        else:
            points = g.integers(-128, 128, (n, d)).astype(np.int8)
    if queries is None:
        if dtype == "u8":
            queries = g.integers(0, 256, (Q, d)).astype(np.uint8)
        else:
            queries = g.integers(-128, 128, (Q, d)).astype(np.int8)
    n, d = points.shape
    Q = queries.shape[0]
    sk = synthdata.gen_secret(N, seed + 3000)
    a = synthdata.gen_uniform_a(P.qs, N, Q * d, seed + 4000).reshape(Q, d, L, N)
    e = synthdata.gen_cbd_error(N, Q * d, seed + 4000).reshape(Q, d, N)
    slot = synthdata.gen_slot_map(n, N, seed + 2000)
    key = synthdata.gen_mask_key(seed + 5000)
    qids = (np.arange(Q, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
            + np.uint64(seed))
    return Problem(P, points, queries, sk, a, e, slot, key, qids)


def workload_problem(w: synthdata.Workload, Q: Optional[int] = None) -> Problem:
    pts = synthdata.gen_points(w)
    qs = synthdata.gen_queries(w, Q)
    return make_problem(w.N, w.L, w.t_bits, 0, 0, 0, seed=w.cid, points=pts, queries=qs)


# ---------------------------------------------------------------- oracle side

def oracle_query_ct(pb: Problem, qi: int) -> np.ndarray:
    return oracle.encrypt_constants(pb.P, pb.sk, pb.a[qi], pb.e[qi],
                                    [int(x) for x in pb.queries[qi]])


def oracle_outputs(pb: Problem, work: Sequence, cts: dict):
    """Full oracle outputs for the (query, chunk) pairs in work."""
    outs, rs = [], []
    for qi, k in work:
        if qi not in cts:
            cts[qi] = oracle_query_ct(pb, qi)
        g, nrm = oracle.chunk_plaintexts(pb.pts, pb.slot, pb.N, k)
        o, r = oracle.server_chunk(pb.P, cts[qi], g, nrm, pb.key, int(pb.qids[qi]), k)
        outs.append(o)
        rs.append(r)
    return np.stack(outs), np.stack(rs)


def true_distances(pb: Problem, qi: int, k: int) -> np.ndarray:
    """||q - p||^2 per slot of chunk k (-1 for padding slots)."""
    ids = pb.slot[k * pb.N:(k + 1) * pb.N]
    out = np.full(pb.N, -1, dtype=np.int64)
    real = ids >= 0
    out[real] = oracle.sqdist(pb.queries[qi], pb.pts[ids[real]])
    return out
