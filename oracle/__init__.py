"""Oracle for the secure k-NN homomorphic distance stage -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does, and the
two implementations share no code: the only thing both consume is the seeded
input module ``synthdata``.

Everything here is the plain definition of what the method computes, in exact
integer arithmetic (Python big integers, and the C loops of ``oracle.c`` for the
quadratic-time negacyclic products):

  parameters      BFV over R_q = Z_q[x]/(x^N+1), q = product of RNS primes
                  q_l = 1 mod 2N, plaintext modulus t, Delta = floor(q/t)
                  (Section 2.3; Section 5, "Parameters")
  encryption      symmetric (private-key) BFV: c1 = a, c0 = -a*s + e + Delta*m,
                  m the constant polynomial q'[i] (Section 2.3; linear-scan
                  protocol, steps 1-2; Section 4.2)
  server product  f_k = sum_i c_i * g_{i,k} with g_{i,k} the coordinate-i
                  plaintext of chunk k taken as -2 p[i] (small signed integers),
                  then the plaintext Delta*[||p||^2 - r]_t added to c0
                  (linear-scan protocol, step 3; Section 4.2)
  decryption      m = round(t (c0 + c1 s mod q) / q) mod t, with the CRT done in
                  big integers; client share = [m + ||q||^2]_t (step 4-5)
  cleartext       squared distances, NaiveTopk (Algorithm 1) and ApproxTopk
                  (Algorithm 2)

Readings of points the paper leaves open are the ones listed in the design
notes (share signs, lift of plaintext coefficients, mask stream, bin
boundaries, ties).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (OpenMP over output coefficients)."""
    if force or not os.path.exists(_SO) or \
            os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_negacyclic_mul.argtypes = [u64p, u64p, ctypes.c_int,
                                            ctypes.c_uint64, u64p]
        L.oracle_inner_coeff.argtypes = [u64p, ctypes.c_int64, i64p,
                                         ctypes.c_int64, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_int]
        L.oracle_inner_coeff.restype = ctypes.c_uint64
        L.oracle_inner_all.argtypes = [u64p, ctypes.c_int64, i64p,
                                       ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_uint64, u64p]
        L.oracle_mul_small.argtypes = [u64p, i64p, ctypes.c_int,
                                       ctypes.c_uint64, u64p]
        L.oracle_chacha20_block.argtypes = [u32p, ctypes.c_uint32, u32p, u32p]
        L.oracle_masks.argtypes = [ctypes.c_char_p, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_int, ctypes.c_int, u32p]
        L.oracle_sample_ternary.argtypes = [ctypes.c_uint64, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_int8)]
        L.oracle_sample_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32,
                                            ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                            u64p]
        L.oracle_sample_cbd21.argtypes = [ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int16)]
        L.oracle_cp_streams.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_int8),
                                        ctypes.POINTER(ctypes.c_int16),
                                        ctypes.POINTER(ctypes.c_int16), u32p]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_sqdist.argtypes = [ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.c_int64, ctypes.c_int, i64p]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Run the OpenMP loops on n threads; returns the count now in effect."""
    lib().oracle_set_threads(int(n))
    return int(lib().oracle_max_threads())


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _p(arr, ct):
    return arr.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------------------
# parameters (Section 2.3; Section 5 "Parameters": N = 2^13, ~180-bit q,
# 128-bit security; the workloads fix N, the number of ~54-bit primes and t)
# ---------------------------------------------------------------------------

def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (first 13 prime bases)."""
    if n < 2:
        return False
    bases = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for p in bases:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def rns_primes(N: int, L: int, bits: int = 54) -> List[int]:
    """The L largest primes below 2^bits with q = 1 mod 2N, descending."""
    m = 2 * N
    c = ((1 << bits) - 1) // m * m + 1
    out = []
    while len(out) < L:
        if is_prime(c):
            out.append(c)
        c -= m
    return out


def plain_modulus(N: int, bits: int) -> int:
    """The smallest prime t >= 2^(bits-1) with t = 1 mod 2N."""
    m = 2 * N
    c = ((1 << (bits - 1)) + m - 1) // m * m + 1
    while not is_prime(c):
        c += m
    return c


# 128-bit-security caps on log2 q for a ternary secret (HE standard tables).
LOGQ_CAP = {1024: 27, 2048: 54, 4096: 109, 8192: 218, 16384: 438, 32768: 881}


class Params:
    def __init__(self, N: int, qs: Sequence[int], t: int):
        self.N, self.qs, self.t = N, list(qs), t
        self.L = len(self.qs)
        self.q = 1
        for x in self.qs:
            self.q *= x
        self.delta = self.q // t

    @classmethod
    def for_workload(cls, N: int, L: int, t_bits: int) -> "Params":
        return cls(N, rns_primes(N, L), plain_modulus(N, t_bits))

    def security_ok(self) -> bool:
        return self.q.bit_length() <= LOGQ_CAP.get(self.N, 0)


# ---------------------------------------------------------------------------
# ring helpers
# ---------------------------------------------------------------------------

def negacyclic_mul(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    """a * b in Z_q[x]/(x^N+1), a, b residues in [0, q) (schoolbook, in C)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().oracle_negacyclic_mul(_p(a, ctypes.c_uint64), _p(b, ctypes.c_uint64),
                                a.size, q, _p(out, ctypes.c_uint64))
    return out


def mul_small(a: np.ndarray, s: np.ndarray, q: int) -> np.ndarray:
    """a * s in Z_q[x]/(x^N+1) with s a small signed integer polynomial."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    s = np.ascontiguousarray(s, dtype=np.int64)
    out = np.empty_like(a)
    lib().oracle_mul_small(_p(a, ctypes.c_uint64), _p(s, ctypes.c_int64),
                           a.size, q, _p(out, ctypes.c_uint64))
    return out


def inner_all(a: np.ndarray, g: np.ndarray, q: int) -> np.ndarray:
    """All coefficients of sum_i a_i * g_i (a: [d][N] residues, g: [d][N]
    small signed integers)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    g = np.ascontiguousarray(g, dtype=np.int64)
    d, N = a.shape
    out = np.empty(N, dtype=np.uint64)
    lib().oracle_inner_all(_p(a, ctypes.c_uint64), N, _p(g, ctypes.c_int64), N,
                           d, N, q, _p(out, ctypes.c_uint64))
    return out


def inner_coeff(a: np.ndarray, g: np.ndarray, q: int, j: int) -> int:
    """Coefficient j of sum_i a_i * g_i."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    g = np.ascontiguousarray(g, dtype=np.int64)
    d, N = a.shape
    return int(lib().oracle_inner_coeff(_p(a, ctypes.c_uint64), N,
                                        _p(g, ctypes.c_int64), N, d, N, q, j))


def small_mod(v: np.ndarray, q: int) -> np.ndarray:
    """Signed small integers taken mod q as residues in [0, q)."""
    v = np.asarray(v, dtype=np.int64)
    return np.where(v < 0, np.uint64(q) - (-v).astype(np.uint64),
                    v.astype(np.uint64)).astype(np.uint64)


# ---------------------------------------------------------------------------
# BFV (symmetric) encryption / decryption
# ---------------------------------------------------------------------------

def encrypt_constants(P: Params, s: np.ndarray, a: np.ndarray, e: np.ndarray,
                      msgs: Sequence[int]) -> np.ndarray:
    """Encrypt each message m_i (taken as [m_i]_t in a constant polynomial).

    s: [N] ternary; a: [d][L][N] uniform residues; e: [d][N] small errors.
    Returns ct [d][2][L][N] uint64 with ct[i][1] = a_i and
    ct[i][0] = -a_i*s + e_i + Delta*m_i  (mod q_l)."""
    d = len(msgs)
    N, L = P.N, P.L
    ct = np.empty((d, 2, L, N), dtype=np.uint64)
    for i in range(d):
        m = int(msgs[i]) % P.t
        for l, ql in enumerate(P.qs):
            as_ = mul_small(a[i, l], s, ql)
            c0 = (small_mod(e[i], ql).astype(object)
                  + (ql - as_.astype(object))) % ql
            c0[0] = (int(c0[0]) + (P.delta % ql) * m) % ql
            ct[i, 0, l] = np.array(c0, dtype=np.uint64)
            ct[i, 1, l] = a[i, l]
    return ct


def sample_secret(seed: int, N: int) -> np.ndarray:
    """Ternary secret key drawn from a seed (ChaCha20 stream, purpose 1)."""
    out = np.empty(N, dtype=np.int8)
    lib().oracle_sample_ternary(seed, N, _p(out, ctypes.c_int8))
    return out


def sample_encryption(P: Params, seed: int, Q: int, d: int
                      ) -> Tuple[np.ndarray, np.ndarray]:
    """Uniform components a [Q][d][L][N] and errors e [Q][d][N] (CBD, eta =
    21) of Q encrypted queries of d coordinates, drawn from a seed (ChaCha20
    streams, purposes 2 and 3, nonce = (query, coordinate, limb))."""
    return _sample_ae(P, seed, Q, d, 2, 3)


def _sample_ae(P: Params, seed: int, Q: int, d: int, pa: int, pe: int):
    N = P.N
    a = np.empty((Q, d, P.L, N), dtype=np.uint64)
    e = np.empty((Q, d, N), dtype=np.int16)
    for qi in range(Q):
        for i in range(d):
            for l, ql in enumerate(P.qs):
                row = np.empty(N, dtype=np.uint64)
                lib().oracle_sample_uniform(seed, pa, qi, i, l, ql, N,
                                            _p(row, ctypes.c_uint64))
                a[qi, i, l] = row
            row = np.empty(N, dtype=np.int16)
            lib().oracle_sample_cbd21(seed, pe, qi, i, N, _p(row, ctypes.c_int16))
            e[qi, i] = row
    return a, e


def sample_public_key(P: Params, s: np.ndarray, seed: int) -> np.ndarray:
    """The client's public key [2][L][N] with its a and e drawn from a seed
    (purposes 4 and 5, nonce (0, 0, limb) and (0, 0, 0))."""
    a, e = _sample_ae(P, seed, 1, 1, 4, 5)
    return public_key(P, s, a[0, 0], e[0, 0])


def phase(P: Params, ct: np.ndarray, s: np.ndarray,
          coeffs: Sequence[int] = None) -> List[int]:
    """x = c0 + c1*s mod q as big integers (CRT over the limbs).

    ct: [2][L][N].  Only the listed coefficients are computed when ``coeffs``
    is given (each coefficient of c1*s is one O(N) sum)."""
    N = P.N
    js = range(N) if coeffs is None else list(coeffs)
    per_limb = []
    for l, ql in enumerate(P.qs):
        if coeffs is None:
            c1s = mul_small(ct[1, l], s, ql)
            vals = [(int(ct[0, l, j]) + int(c1s[j])) % ql for j in js]
        else:
            s2 = np.asarray(s, dtype=np.int64)[None, :]
            vals = [(int(ct[0, l, j]) + inner_coeff(ct[1, l][None, :], s2, ql, j))
                    % ql for j in js]
        per_limb.append(vals)
    out = []
    for n in range(len(js)):
        x = 0
        for l, ql in enumerate(P.qs):
            Ml = P.q // ql
            x += per_limb[l][n] * Ml * pow(Ml, -1, ql)
        out.append(x % P.q)
    return out


def decrypt(P: Params, ct: np.ndarray, s: np.ndarray,
            coeffs: Sequence[int] = None) -> List[int]:
    """m_j = floor((t x_j + floor(q/2)) / q) mod t."""
    return [((P.t * x + P.q // 2) // P.q) % P.t for x in phase(P, ct, s, coeffs)]


def noise(P: Params, ct: np.ndarray, s: np.ndarray, msg: Sequence[int],
          coeffs: Sequence[int] = None) -> List[int]:
    """Centred v_j = [x_j - Delta*m_j]_q for the expected plaintext m."""
    out = []
    for x, m in zip(phase(P, ct, s, coeffs), msg):
        v = (x - P.delta * (int(m) % P.t)) % P.q
        if v > P.q // 2:
            v -= P.q
        out.append(v)
    return out


# ---------------------------------------------------------------------------
# the server's distance stage
# ---------------------------------------------------------------------------

def chunk_plaintexts(points: np.ndarray, slot_pt: np.ndarray, N: int,
                     k: int) -> Tuple[np.ndarray, np.ndarray]:
    """g_{i,k}[j] = -2 p[i] for the point in slot j of chunk k (0 for padding),
    as signed integers [d][N]; and ||p||^2 per slot [N]."""
    ids = slot_pt[k * N:(k + 1) * N]
    d = points.shape[1]
    g = np.zeros((d, N), dtype=np.int64)
    nrm = np.zeros(N, dtype=np.int64)
    real = ids >= 0
    pv = points[ids[real]].astype(np.int64)
    g[:, real] = -2 * pv.T
    nrm[real] = (pv * pv).sum(axis=1)
    return g, nrm


def chunk_plaintexts_shares(shares: np.ndarray, norm_shares: np.ndarray, slot_pt: np.ndarray,
                            N: int, k: int, t: int) -> Tuple[np.ndarray, np.ndarray]:
    """Plaintexts of chunk k when the server holds only additive shares p_s
    (mod t) of the points and of their squared norms (Section 4.2, last
    paragraph): g_{i,k}[j] = the representative of -2 p_s[i] mod t in
    (-t/2, t/2] (0 for padding) and the norm plane = the norm share."""
    ids = slot_pt[k * N:(k + 1) * N]
    d = shares.shape[1]
    g = np.zeros((d, N), dtype=np.int64)
    nrm = np.zeros(N, dtype=np.int64)
    real = ids >= 0
    ps = shares[ids[real]].astype(np.int64)
    v = (-2 * ps) % t
    v = np.where(v > t // 2, v - t, v)
    g[:, real] = v.T
    nrm[real] = norm_shares[ids[real]].astype(np.int64)
    return g, nrm


def masks(key: bytes, query_id: int, chunk: int, t: int, N: int,
          j0: int = 0, cnt: int = None) -> np.ndarray:
    cnt = N - j0 if cnt is None else cnt
    out = np.empty(cnt, dtype=np.uint32)
    lib().oracle_masks(key, query_id, chunk, t, j0, cnt,
                       _p(out, ctypes.c_uint32))
    return out


def server_chunk(P: Params, ct: np.ndarray, g: np.ndarray, nrm: np.ndarray,
                 key: bytes, query_id: int, chunk: int
                 ) -> Tuple[np.ndarray, np.ndarray]:
    """Full output of one (query, chunk): ciphertext [2][L][N] and server
    share r [N].  f = sum_i c_i * g_i;  c0 += Delta * [||p||^2 - r]_t."""
    N, L = P.N, P.L
    out = np.empty((2, L, N), dtype=np.uint64)
    r = masks(key, query_id, chunk, P.t, N)
    mval = (nrm - r.astype(np.int64)) % P.t
    for l, ql in enumerate(P.qs):
        for c in range(2):
            out[c, l] = inner_all(ct[:, c, l, :], g, ql)
        dl = P.delta % ql
        add = np.array([(int(x) * dl) % ql for x in mval], dtype=object)
        out[0, l] = np.array((out[0, l].astype(object) + add) % ql,
                             dtype=np.uint64)
    return out, r


def server_coeffs(P: Params, ct: np.ndarray, g: np.ndarray, nrm: np.ndarray,
                  key: bytes, query_id: int, chunk: int, js: Sequence[int]
                  ) -> Tuple[np.ndarray, np.ndarray]:
    """Sampled coefficients js of server_chunk: ciphertext [2][L][len(js)] and
    the server shares at js."""
    L = P.L
    out = np.empty((2, L, len(js)), dtype=np.uint64)
    r = np.array([masks(key, query_id, chunk, P.t, P.N, j, 1)[0] for j in js],
                 dtype=np.uint32)
    for n, j in enumerate(js):
        mval = (int(nrm[j]) - int(r[n])) % P.t
        for l, ql in enumerate(P.qs):
            for c in range(2):
                v = inner_coeff(ct[:, c, l, :], g, ql, j)
                if c == 0:
                    v = (v + (P.delta % ql) * mval) % ql
                out[c, l, n] = v
    return out, r


def client_shares(P: Params, ct_out: np.ndarray, s: np.ndarray, qnorm2: int,
                  coeffs: Sequence[int] = None) -> np.ndarray:
    """Client share [Dec(f) + ||q||^2]_t for one output ciphertext."""
    m = decrypt(P, ct_out, s, coeffs)
    return np.array([(x + qnorm2) % P.t for x in m], dtype=np.uint32)


# ---------------------------------------------------------------------------
# circuit privacy: re-randomisation and noise flooding (Section 2.3: the AHE
# must hide the server's computation, by noise flooding; Section 5
# "Parameters": statistical circuit privacy)
# ---------------------------------------------------------------------------

def public_key(P: Params, s: np.ndarray, a: np.ndarray, e: np.ndarray) -> np.ndarray:
    """The client's public key [2][L][N]: p1 = a, p0 = -a*s + e (mod q_l),
    an encryption of zero.  a: [L][N] uniform residues, e: [N] small errors."""
    return encrypt_constants(P, s, a[None], e[None], [0])[0]


def flood_bits(P: Params) -> int:
    """Default width b of the flooding noise, uniform in [-2^b, 2^b): the
    largest b with 2^b <= Delta / 4, so that the flood takes at most a quarter
    of the decryption margin Delta / 2."""
    return P.delta.bit_length() - 3


def cp_randomness(P: Params, key: bytes, query_id: int, chunk: int, b: int):
    """u (ternary), e1, e2 (CBD, eta = 21) and the flood integers
    X_j mod 2^(b+1) - 2^b of one output, from the server's key."""
    N = P.N
    u = np.empty(N, dtype=np.int8)
    e1 = np.empty(N, dtype=np.int16)
    e2 = np.empty(N, dtype=np.int16)
    words = np.empty((N, 8), dtype=np.uint32)
    lib().oracle_cp_streams(key, query_id, chunk, N, _p(u, ctypes.c_int8),
                            _p(e1, ctypes.c_int16), _p(e2, ctypes.c_int16),
                            _p(words, ctypes.c_uint32))
    flood = []
    for j in range(N):
        X = 0
        for w in reversed(words[j]):
            X = (X << 32) | int(w)
        flood.append((X % (1 << (b + 1))) - (1 << b))
    return u, e1, e2, flood


def rerandomize(P: Params, f: np.ndarray, pk: np.ndarray, key: bytes, query_id: int,
                chunk: int, b: int) -> np.ndarray:
    """f + (p0 u + e1 + flood, p1 u + e2) for one output ciphertext f
    [2][L][N]: a fresh encryption of zero under the client's public key
    (re-randomises both components) plus noise flooding in c0."""
    u, e1, e2, flood = cp_randomness(P, key, query_id, chunk, b)
    out = np.empty_like(f)
    for l, ql in enumerate(P.qs):
        pu0 = mul_small(pk[0, l], u, ql).astype(object)
        pu1 = mul_small(pk[1, l], u, ql).astype(object)
        c0 = [(int(f[0, l, j]) + int(pu0[j]) + int(e1[j]) + flood[j]) % ql
              for j in range(P.N)]
        c1 = [(int(f[1, l, j]) + int(pu1[j]) + int(e2[j])) % ql for j in range(P.N)]
        out[0, l] = np.array(c0, dtype=np.uint64)
        out[1, l] = np.array(c1, dtype=np.uint64)
    return out


# ---------------------------------------------------------------------------
# cleartext: distances and top-k (Algorithms 1 and 2)
# ---------------------------------------------------------------------------

def sqdist(query: np.ndarray, points: np.ndarray) -> np.ndarray:
    qv = np.ascontiguousarray(query, dtype=np.int32)
    pv = np.ascontiguousarray(points, dtype=np.int32)
    out = np.empty(pv.shape[0], dtype=np.int64)
    lib().oracle_sqdist(_p(qv, ctypes.c_int32), _p(pv, ctypes.c_int32),
                        pv.shape[0], pv.shape[1], _p(out, ctypes.c_int64))
    return out


def naive_topk(vals: Sequence[int], ids: Sequence[int], k: int
               ) -> Tuple[List[int], List[int]]:
    """Algorithm 1's selection: the k smallest values in ascending order with
    their IDs.  Ties are read as a stable selection (an earlier position
    comes first): the output is the k smallest (value, position) pairs.
    Positions past the input are (infinity, -1)."""
    order = sorted(range(len(vals)), key=lambda j: (vals[j], j))[:k]
    out_v = [vals[j] for j in order] + [float("inf")] * (k - len(order))
    out_i = [ids[j] for j in order] + [-1] * (k - len(order))
    return out_v, out_i


def bin_bounds(n: int, l: int) -> List[Tuple[int, int]]:
    """l consecutive bins over n items; when l does not divide n the first
    n mod l bins take one extra item."""
    base, extra = divmod(n, l)
    out, s = [], 0
    for i in range(l):
        e = s + base + (1 if i < extra else 0)
        out.append((s, e))
        s = e
    return out


def approx_topk(vals: np.ndarray, ids: np.ndarray, k: int, l: int
                ) -> Tuple[List[int], List[int]]:
    """Algorithm 2: per-bin minimum (first occurrence), then Algorithm 1 on
    the l bin minima.  The input is already in the server's random order."""
    if k > l:
        raise ValueError("k must not exceed l")
    mins, mids = [], []
    for s, e in bin_bounds(len(vals), l):
        j = s + int(np.argmin(vals[s:e]))
        mins.append(int(vals[j]))
        mids.append(int(ids[j]))
    return naive_topk(mins, mids, k)
