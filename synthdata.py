"""Seeded synthetic inputs for the secure k-NN distance stage.

This module only draws random numbers and shapes them; it holds none of the
method's arithmetic (no encryption, no ring products, no distances).  It is the
one source of inputs shared by the oracle, the tests, the benchmark and the
serving loop, so both sides of every parity check see the same bytes.

The real datasets the paper evaluates on (SIFT, Deep1B, Amazon; Section 5,
"Datasets") are not available here.  Each workload below is a synthetic stand-in
with the shape, coordinate width and value structure the paper describes for
those datasets (n, d, 8-bit coordinates), as restated in the workload table.

Randomness the method itself draws is produced here and passed in as inputs:
  * the client's ternary secret key s,
  * the uniform ciphertext component a (one polynomial per RNS limb),
  * the centred-binomial error e,
  * the server's random permutation of its points.
The server's masks are the one exception: they are drawn inside the hot path
from ChaCha20 (RFC 8439), which both sides implement independently; this
module only supplies the 256-bit key.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

# Seeds: data, perm, sk, enc, mask, arrivals = base + config number.
SEED_DATA, SEED_PERM, SEED_SK, SEED_ENC, SEED_MASK, SEED_ARR = (
    1000, 2000, 3000, 4000, 5000, 6000)


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape of one synthetic workload (no arithmetic, just sizes and rules)."""
    cid: int
    name: str
    n: int                 # database points
    d: int                 # dimensions
    dtype: str             # "u8" or "i8"
    gen: str               # point generator name
    N: int                 # ring degree
    L: int                 # RNS limbs
    t_bits: int            # t = smallest prime >= 2^(t_bits-1), t = 1 mod 2N
    k: int                 # neighbours returned
    l: int                 # bins of the approximate top-k (0 = unused)
    Q: int                 # queries per launch
    mode: str              # plain | fused | batched | clustered | serving


WORKLOADS: Dict[int, Workload] = {
    1: Workload(1, "linear-scan 10K x 128 u8, N=4096, L=2", 10_000, 128, "u8",
                "uniform_u8", 4096, 2, 25, 10, 100, 1, "plain"),
    2: Workload(2, "linear-scan 1M x 128 u8 (Gaussian mixture), N=8192, L=3",
                1_000_000, 128, "u8", "mixture_u8", 8192, 3, 25, 10, 1000, 1,
                "plain"),
    3: Workload(3, "batched 64 queries, 1M x 96 i8 (unit-norm x127), N=8192, L=3",
                1_000_000, 96, "i8", "unitnorm_i8", 8192, 3, 26, 10, 1000, 64,
                "batched"),
    4: Workload(4, "clustered 10M x 96 i8, 16384 Zipf clusters + 1% stash, "
                "32 queries x 64 clusters, N=8192, L=3",
                10_000_000, 96, "i8", "zipf_clusters_i8", 8192, 3, 26, 10, 0,
                32, "clustered"),
    5: Workload(5, "serving over three resident databases, N=8192, L=3",
                0, 0, "mixed", "serving", 8192, 3, 26, 10, 0, 0, "serving"),
}

# The batched benchmark row: workload 2's database (1M x 128 u8) with 64 queries.
BATCHED_1M128 = dataclasses.replace(
    WORKLOADS[2], name="batched 64 queries, 1M x 128 u8 (Gaussian mixture)",
    Q=64, mode="batched")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# database / query generators
# --------------------------------------------------------------------------

def _uniform_u8(g: np.random.Generator, n: int, d: int) -> np.ndarray:
    return g.integers(0, 256, size=(n, d), dtype=np.uint8)


def _mixture_centers(d: int, seed: int, n_comp: int = 1000) -> np.ndarray:
    return rng(seed * 7 + 1).uniform(0.0, 255.0, size=(n_comp, d))


def _mixture_u8(g: np.random.Generator, n: int, d: int, centers: np.ndarray,
                sigma: float = 20.0, block: int = 65536) -> np.ndarray:
    out = np.empty((n, d), dtype=np.uint8)
    for s in range(0, n, block):
        e = min(n, s + block)
        comp = g.integers(0, centers.shape[0], size=e - s)
        x = centers[comp] + g.normal(0.0, sigma, size=(e - s, d))
        out[s:e] = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    return out


def _unitnorm_i8(g: np.random.Generator, n: int, d: int,
                 block: int = 65536) -> np.ndarray:
    out = np.empty((n, d), dtype=np.int8)
    for s in range(0, n, block):
        e = min(n, s + block)
        x = g.normal(0.0, 1.0, size=(e - s, d))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[s:e] = np.clip(np.rint(x * 127.0), -127, 127).astype(np.int8)
    return out


def gen_points(w: Workload, n: Optional[int] = None, seed: Optional[int] = None
               ) -> np.ndarray:
    """Database points [n][d] (uint8 or int8) for workload ``w``."""
    n = w.n if n is None else n
    seed = SEED_DATA + w.cid if seed is None else seed
    g = rng(seed)
    if w.gen == "uniform_u8":
        return _uniform_u8(g, n, w.d)
    if w.gen == "mixture_u8":
        return _mixture_u8(g, n, w.d, _mixture_centers(w.d, seed))
    if w.gen == "unitnorm_i8":
        return _unitnorm_i8(g, n, w.d)
    raise ValueError(f"gen_points: no flat generator for {w.gen}")


def gen_queries(w: Workload, Q: Optional[int] = None,
                seed: Optional[int] = None) -> np.ndarray:
    """Queries [Q][d] drawn from the same distribution as the points."""
    Q = max(1, w.Q) if Q is None else Q
    seed = SEED_DATA + w.cid if seed is None else seed
    g = rng(seed + 500_000)
    if w.gen == "uniform_u8":
        return _uniform_u8(g, Q, w.d)
    if w.gen == "mixture_u8":
        return _mixture_u8(g, Q, w.d, _mixture_centers(w.d, seed))
    if w.gen in ("unitnorm_i8", "zipf_clusters_i8"):
        return _unitnorm_i8(g, Q, w.d)
    raise ValueError(w.gen)


# --------------------------------------------------------------------------
# randomness the method draws (passed in to both sides)
# --------------------------------------------------------------------------

def gen_secret(N: int, seed: int) -> np.ndarray:
    """Ternary secret key, uniform over {-1, 0, 1}^N (int8)."""
    return (rng(seed).integers(0, 3, size=N, dtype=np.int64) - 1).astype(np.int8)


def gen_uniform_a(qs: List[int], N: int, count: int, seed: int) -> np.ndarray:
    """Uniform ciphertext components: uint64 [count][L][N], limb l uniform in
    [0, q_l).  By the CRT this is a uniform element of R_q per polynomial."""
    g = rng(seed)
    out = np.empty((count, len(qs), N), dtype=np.uint64)
    for l, q in enumerate(qs):
        out[:, l, :] = g.integers(0, q, size=(count, N), dtype=np.uint64)
    return out


def gen_cbd_error(N: int, count: int, seed: int, eta: int = 21) -> np.ndarray:
    """Centred binomial error CBD_eta (variance eta/2): int16 [count][N]."""
    g = rng(seed + 1)
    return (g.binomial(2 * eta, 0.5, size=(count, N)) - eta).astype(np.int16)


def gen_perm(n: int, seed: int) -> np.ndarray:
    """The server's uniformly random permutation of its n points (int64)."""
    return rng(seed).permutation(n).astype(np.int64)


def gen_slot_map(n: int, N: int, seed: int) -> np.ndarray:
    """The server's random placement of n points into ceil(n/N) chunks of N
    slots: slot s of chunk k holds point perm[kN + s] (perm = gen_perm(n,
    seed)); the padding slots of the last chunk hold -1.  int64 [C N]."""
    C = (n + N - 1) // N
    out = np.full(C * N, -1, dtype=np.int64)
    out[:n] = gen_perm(n, seed)
    return out


def gen_mask_key(seed: int) -> bytes:
    """256-bit key of the server's mask stream."""
    return rng(seed).integers(0, 256, size=32, dtype=np.uint8).tobytes()


# --------------------------------------------------------------------------
# clustered workload (Zipf cluster sizes, stash)
# --------------------------------------------------------------------------

def zipf_cluster_sizes(n_clusters: int = 16384, total: int = 9_900_000,
                       s: float = 1.1, min_size: int = 50) -> np.ndarray:
    """size_r = max(min_size, round(C r^-s)), C chosen so the sizes sum to
    ``total`` (the last cluster absorbs the rounding residue)."""
    r = np.arange(1, n_clusters + 1, dtype=np.float64)

    def sizes(C):
        return np.maximum(min_size, np.rint(C * r ** (-s))).astype(np.int64)

    lo, hi = 1.0, float(total)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sizes(mid).sum() < total:
            lo = mid
        else:
            hi = mid
    out = sizes(lo)
    out[0] += total - out.sum()
    return out


@dataclasses.dataclass
class ClusteredDB:
    points: np.ndarray          # [n][d] int8, clusters contiguous then stash
    cluster_sizes: np.ndarray   # [n_clusters] int64
    centers: np.ndarray         # [n_clusters][d] int8 (quantised centres)
    stash_size: int


def gen_clustered(n_clusters: int = 16384, total_clustered: int = 9_900_000,
                  stash: int = 100_000, d: int = 96, sigma_c: float = 0.25,
                  seed: int = SEED_DATA + 4, block: int = 1 << 18) -> ClusteredDB:
    g = rng(seed)
    sizes = zipf_cluster_sizes(n_clusters, total_clustered)
    cen = g.normal(0.0, 1.0, size=(n_clusters, d))
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    n = int(sizes.sum()) + stash
    pts = np.empty((n, d), dtype=np.int8)
    owner = np.concatenate([np.repeat(np.arange(n_clusters), sizes),
                            g.integers(0, n_clusters, size=stash)])
    cen32 = cen.astype(np.float32)
    for s in range(0, n, block):
        e = min(n, s + block)
        x = cen32[owner[s:e]] + np.float32(sigma_c) * g.standard_normal(
            size=(e - s, d), dtype=np.float32)
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        pts[s:e] = np.clip(np.rint(x * np.float32(127.0)), -127, 127).astype(np.int8)
    qc = np.clip(np.rint(cen * 127.0), -127, 127).astype(np.int8)
    return ClusteredDB(pts, sizes, qc, stash)


# --------------------------------------------------------------------------
# serving workload (Poisson arrivals)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    db: int          # which resident database
    Q: int           # queries in the request
    k: int


def gen_arrivals(n_req: int, rate_per_s: float, n_dbs: int = 3,
                 max_q: int = 64, seed: int = SEED_ARR + 5) -> List[Request]:
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_per_s, size=n_req)
    t = np.cumsum(gaps)
    dbs = g.integers(0, n_dbs, size=n_req)
    qs = g.integers(1, max_q + 1, size=n_req)
    ks = g.choice(np.array([1, 10, 100]), size=n_req)
    return [Request(i, float(t[i]), int(dbs[i]), int(qs[i]), int(ks[i]))
            for i in range(n_req)]
