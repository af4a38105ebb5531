"""Cleartext reference of the selection that follows the distance stage.

In the protocol the two parties feed their shares to a garbled circuit that
computes the approximate top-k (functionality F_aTOPk; Algorithm 2) or the
exact top-k (F_TOPk; Algorithm 1).  The garbled circuit is out of scope; this
module computes the same selection in the clear from the reconstructed
distances, for checking, recall measurement and the serving loop.

* reconstruct(): d = [client + server]_t, then floor(d / 2^r) (the optional
  truncation of Section 3 "Approximate Distances").
* naive_topk(): Algorithm 1's selection -- the k smallest values in
  ascending order, equal values in input order.
* approx_topk(): Algorithm 2 -- l consecutive bins over the (already
  randomly permuted) list, the first minimum of each bin, then Algorithm 1 on
  the l bin minima.  When l does not divide n the first n mod l bins take one
  extra item.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def reconstruct(client_share: np.ndarray, server_share: np.ndarray, t: int,
                r_bits: int = 0) -> np.ndarray:
    """Squared distances from additive shares mod t (int64)."""
    d = (np.asarray(client_share, dtype=np.int64) +
         np.asarray(server_share, dtype=np.int64)) % int(t)
    return d >> r_bits if r_bits else d


def naive_topk(values: np.ndarray, ids: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 1's selection on (values, ids): (k values ascending, their
    ids), equal values in input order; missing entries (k > n) are
    (max int64, -1)."""
    values = np.asarray(values, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    out_v = np.full(k, np.iinfo(np.int64).max, dtype=np.int64)
    out_i = np.full(k, -1, dtype=np.int64)
    n = len(values)
    kk = min(k, n)
    if kk:
        if kk < n:
            # the k-th smallest value in linear time; every smaller value, then
            # the first of the equal ones in input order
            thr = np.partition(values, kk - 1)[kk - 1]
            below = np.flatnonzero(values < thr)
            eq = np.flatnonzero(values == thr)[:kk - len(below)]
            sel = np.sort(np.concatenate([below, eq]))
        else:
            sel = np.arange(n)
        o = sel[np.argsort(values[sel], kind="stable")]
        out_v[:kk], out_i[:kk] = values[o], ids[o]
    return out_v, out_i


def bin_edges(n: int, l: int) -> np.ndarray:
    base, extra = divmod(n, l)
    sizes = np.full(l, base, dtype=np.int64)
    sizes[:extra] += 1
    return np.concatenate([[0], np.cumsum(sizes)])


def approx_topk(values: np.ndarray, ids: np.ndarray, k: int, l: int
                ) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 2: first minimum of each of l bins, then Algorithm 1."""
    if k > l:
        raise ValueError("approx_topk needs k <= l")
    values = np.asarray(values, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    n = len(values)
    if l > n:
        raise ValueError("approx_topk needs l <= n")
    edges = bin_edges(n, l)
    if n % l == 0:
        b = n // l
        arg = values.reshape(l, b).argmin(axis=1) + np.arange(l) * b
    else:
        arg = np.array([edges[i] + int(np.argmin(values[edges[i]:edges[i + 1]]))
                        for i in range(l)], dtype=np.int64)
    return naive_topk(values[arg], ids[arg], k)


def recall(found_ids: np.ndarray, true_ids: np.ndarray) -> float:
    """|found & true| / |true| (the k-NN accuracy measure of Section 5)."""
    t = set(int(x) for x in true_ids if x >= 0)
    return len(t & set(int(x) for x in found_ids if x >= 0)) / max(1, len(t))
