"""Pins of the oracle against things other than itself (CPU only).

Each check is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a wrong constant) fails it:
published test vectors, an independent library routine, brute force on tiny
inputs, closed forms and the exact decryption identities of the scheme.
"""
import ctypes
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synthdata

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- ChaCha20

def _read_hex(name):
    with open(os.path.join(GOLD, name)) as f:
        return bytes.fromhex("".join(l.strip() for l in f
                                     if l.strip() and not l.startswith("#")))


def _block(key: bytes, counter: int, nonce: bytes) -> bytes:
    kw = (ctypes.c_uint32 * 8)(*np.frombuffer(key, dtype="<u4").tolist())
    nw = (ctypes.c_uint32 * 3)(*np.frombuffer(nonce, dtype="<u4").tolist())
    out = (ctypes.c_uint32 * 16)()
    oracle.lib().oracle_chacha20_block(kw, counter, nw, out)
    return np.array(list(out), dtype="<u4").tobytes()


def test_chacha20_rfc8439_block_vector():
    # RFC 8439 Section 2.3.2
    key = bytes(range(32))
    nonce = bytes([0, 0, 0, 9, 0, 0, 0, 0x4a, 0, 0, 0, 0])
    assert _block(key, 1, nonce) == _read_hex("chacha20_rfc8439_s2_3_2.txt")


def _openssl_keystream(key, counter, nonce, nbytes):
    try:
        lc = ctypes.CDLL("libcrypto.so.3")
    except OSError:
        pytest.skip("libcrypto not available")
    lc.EVP_CIPHER_CTX_new.restype = ctypes.c_void_p
    lc.EVP_chacha20.restype = ctypes.c_void_p
    lc.EVP_EncryptInit_ex.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_char_p] * 2
    lc.EVP_EncryptUpdate.argtypes = [ctypes.c_void_p, ctypes.c_char_p,
                                     ctypes.POINTER(ctypes.c_int),
                                     ctypes.c_char_p, ctypes.c_int]
    lc.EVP_CIPHER_CTX_free.argtypes = [ctypes.c_void_p]
    ctx = lc.EVP_CIPHER_CTX_new()
    iv = counter.to_bytes(4, "little") + nonce
    assert lc.EVP_EncryptInit_ex(ctx, lc.EVP_chacha20(), None, key, iv) == 1
    out = ctypes.create_string_buffer(nbytes)
    ol = ctypes.c_int(0)
    assert lc.EVP_EncryptUpdate(ctx, out, ctypes.byref(ol), b"\0" * nbytes,
                                nbytes) == 1
    lc.EVP_CIPHER_CTX_free(ctx)
    return out.raw[:ol.value]


def test_chacha20_matches_openssl_keystream():
    g = np.random.default_rng(7)
    for _ in range(5):
        key = g.integers(0, 256, 32, dtype=np.uint8).tobytes()
        nonce = g.integers(0, 256, 12, dtype=np.uint8).tobytes()
        ctr = int(g.integers(0, 1 << 31))
        ks = _openssl_keystream(key, ctr, nonce, 64 * 3)
        ours = b"".join(_block(key, ctr + b, nonce) for b in range(3))
        assert ours == ks


def test_mask_stream_definition():
    """Mask j = (128-bit LE integer of words 4(j%4).. of block j//4) mod t,
    nonce = (query id lo, query id hi, chunk); recomputed from the OpenSSL
    keystream."""
    key = synthdata.gen_mask_key(99)
    qid, chunk, t, N = (5 << 32) + 17, 3, 16957441, 64
    nonce = np.array([qid & 0xffffffff, qid >> 32, chunk], dtype="<u4").tobytes()
    ks = _openssl_keystream(key, 0, nonce, N * 16)
    want = [int.from_bytes(ks[16 * j:16 * j + 16], "little") % t
            for j in range(N)]
    got = oracle.masks(key, qid, chunk, t, N)
    assert got.tolist() == want
    sub = oracle.masks(key, qid, chunk, t, N, 13, 7)
    assert sub.tolist() == want[13:20]


# ---------------------------------------------------------------- parameters

def _trial_division_prime(p: int) -> bool:
    r = math.isqrt(p)
    if p % 2 == 0:
        return p == 2
    for s in range(3, r + 1, 1 << 24):
        cand = np.arange(s, min(r + 1, s + (1 << 24)), 2, dtype=np.int64)
        if np.any(p % cand == 0):
            return False
    return True


@pytest.mark.parametrize("N,L,want", [
    (4096, 2, [0x3ffffffffd6001, 0x3ffffffffd2001]),
    (8192, 3, [0x3fffffffef8001, 0x3fffffffeb8001, 0x3fffffffe7c001]),
])
def test_rns_primes_are_the_largest(N, L, want):
    got = oracle.rns_primes(N, L)
    assert got == want
    for q in got:
        assert q % (2 * N) == 1 and q < (1 << 54)
        assert _trial_division_prime(q)
    # every other candidate = 1 mod 2N between the smallest prime and 2^54 is
    # composite, shown by a Fermat witness
    c = ((1 << 54) - 1) // (2 * N) * (2 * N) + 1
    while c >= got[-1]:
        if c not in got:
            assert any(pow(a, c - 1, c) != 1 for a in (2, 3, 5, 7))
        c -= 2 * N


@pytest.mark.parametrize("N,bits,want", [(4096, 25, 16801793),
                                         (8192, 25, 16957441),
                                         (8192, 26, 33832961)])
def test_plain_modulus(N, bits, want):
    t = oracle.plain_modulus(N, bits)
    assert t == want and t % (2 * N) == 1 and t.bit_length() == bits
    assert _trial_division_prime(t)
    c = (1 << (bits - 1)) + 1
    while c < t:
        if c % (2 * N) == 1:
            assert any(pow(a, c - 1, c) != 1 for a in (2, 3, 5, 7))
        c += 1


def _golden_caps():
    caps = {}
    for line in open(os.path.join(GOLD, "he_standard_128bit_ternary.txt")):
        if line.strip() and not line.startswith("#"):
            n, b = line.split()
            caps[int(n)] = int(b)
    return caps


def test_security_check_matches_he_standard_caps():
    """Params.security_ok accepts exactly the moduli within the standard's
    128-bit caps: at every tabulated N a modulus of the cap's bit length
    passes and one bit more fails; degrees outside the table fail."""
    caps = _golden_caps()
    assert sorted(caps) == [1024, 2048, 4096, 8192, 16384, 32768]
    for N, b in caps.items():
        at = oracle.Params(N, [(1 << (b - 1)) + 1], 3)
        over = oracle.Params(N, [(1 << b) + 1], 3)
        assert at.q.bit_length() == b and at.security_ok(), N
        assert over.q.bit_length() == b + 1 and not over.security_ok(), N
        # split over several limbs the same way
        two = oracle.Params(N, [(1 << (b // 2)) + 1, (1 << (b - b // 2 - 1)) + 1], 3)
        assert two.q.bit_length() == b and two.security_ok(), N
    for N in (16, 512, 3000, 65536):
        assert not oracle.Params(N, [(1 << 20) + 1], 3).security_ok(), N
    # the paper's own parameter set (N = 2^13, 180-bit q) is within its cap;
    # the same q at N = 4096 is not
    q180 = [(1 << 59) + 1, (1 << 59) + 3, (1 << 61) + 1]
    assert oracle.Params(8192, q180, 1 << 23).q.bit_length() == 180
    assert oracle.Params(8192, q180, 1 << 23).security_ok()
    assert not oracle.Params(4096, q180, 1 << 23).security_ok()


def test_workload_params_secure_and_wide_enough():
    for w in [synthdata.WORKLOADS[c] for c in (1, 2, 3)]:
        P = oracle.Params.for_workload(w.N, w.L, w.t_bits)
        assert P.security_ok()
        maxdiff = 255 if w.dtype == "u8" else 254
        # the bit-width rule b_d = 2 b_c + ceil(log2 d): every distance < t
        assert w.d * maxdiff ** 2 < P.t
        assert P.delta == P.q // P.t


# ---------------------------------------------------------------- ring

def _negacyclic_bigint(a, b, q):
    """Dense integer product, then x^N = -1 (an independent route)."""
    N = len(a)
    full = [0] * (2 * N)
    for u in range(N):
        for v in range(N):
            full[u + v] += int(a[u]) * int(b[v])
    return [(full[j] - full[j + N]) % q for j in range(N)]


@pytest.mark.parametrize("N", [1, 2, 16, 64])
def test_negacyclic_mul_brute_force(N):
    q = oracle.rns_primes(max(N, 2), 1)[0]
    g = np.random.default_rng(N)
    a = g.integers(0, q, N, dtype=np.uint64)
    b = g.integers(0, q, N, dtype=np.uint64)
    assert oracle.negacyclic_mul(a, b, q).tolist() == _negacyclic_bigint(a, b, q)
    s = g.integers(-600, 600, N)
    assert oracle.mul_small(a, s, q).tolist() == \
        _negacyclic_bigint(a, oracle.small_mod(s, q), q)


def test_negacyclic_monomial_is_signed_rotation():
    N, q = 32, oracle.rns_primes(32, 1)[0]
    a = np.random.default_rng(1).integers(0, q, N, dtype=np.uint64)
    for j in (0, 1, 5, 31):
        mono = np.zeros(N, dtype=np.int64)
        mono[j] = 1
        got = oracle.mul_small(a, mono, q)
        want = [int(a[(u - j) % N]) if u >= j else (q - int(a[u - j + N])) % q
                for u in range(N)]
        assert got.tolist() == want


def test_inner_is_sum_of_products():
    N, d, q = 64, 5, oracle.rns_primes(64, 1)[0]
    g = np.random.default_rng(3)
    a = g.integers(0, q, (d, N), dtype=np.uint64)
    gg = g.integers(-510, 1, (d, N))
    want = [0] * N
    for i in range(d):
        p = _negacyclic_bigint(a[i], oracle.small_mod(gg[i], q), q)
        want = [(x + y) % q for x, y in zip(want, p)]
    assert oracle.inner_all(a, gg, q).tolist() == want
    for j in (0, 17, 63):
        assert oracle.inner_coeff(a, gg, q, j) == want[j]


# ---------------------------------------------------------------- BFV

def _toy_params(N=16, L=2, t=257):
    return oracle.Params(N, oracle.rns_primes(N, L), t)


@pytest.mark.parametrize("t", [257, 256])
def test_decrypt_of_encrypt_exhaustive_small(t):
    """Dec(Enc(m)) = m for every m in Z_t, and a fresh ciphertext's noise is
    exactly its error polynomial (c0 + c1 s = e + Delta m); for a prime t and
    for t a power of two (the paper's choice, Section 5)."""
    P = _toy_params(t=t)
    s = synthdata.gen_secret(P.N, 1)
    msgs = list(range(P.t))
    a = synthdata.gen_uniform_a(P.qs, P.N, len(msgs), 2)
    e = synthdata.gen_cbd_error(P.N, len(msgs), 3)
    ct = oracle.encrypt_constants(P, s, a, e, msgs)
    for i, m in enumerate(msgs):
        dec = oracle.decrypt(P, ct[i], s)
        assert dec[0] == m and all(x == 0 for x in dec[1:])
        assert oracle.noise(P, ct[i], s, [m] + [0] * (P.N - 1)) == \
            [int(x) for x in e[i]]


def test_decrypt_sampled_coeffs_agree_with_full():
    P = _toy_params(N=64, L=3, t=oracle.plain_modulus(64, 20))
    s = synthdata.gen_secret(P.N, 4)
    a = synthdata.gen_uniform_a(P.qs, P.N, 1, 5)
    e = synthdata.gen_cbd_error(P.N, 1, 6)
    ct = oracle.encrypt_constants(P, s, a, e, [12345])
    full = oracle.phase(P, ct[0], s)
    js = [0, 7, 63]
    assert oracle.phase(P, ct[0], s, js) == [full[j] for j in js]


def test_encoding_identity_plaintext():
    """Section 4.2: sum_i f_i g_i = sum_j <q, p_j> x^j in Z_t[x]/(x^N+1) when
    f_i is the constant q[i] and g_i carries coordinate i of every point."""
    N, d, t = 32, 6, 65537
    g = np.random.default_rng(11)
    pts = g.integers(0, 256, (N, d))
    qv = g.integers(0, 256, d)
    acc = [0] * N
    for i in range(d):
        f = [int(qv[i])] + [0] * (N - 1)
        gi = [int(pts[j, i]) for j in range(N)]
        acc = [(x + y) % t for x, y in zip(acc, _negacyclic_bigint(f, gi, t))]
    assert acc == [int(pts[j] @ qv) % t for j in range(N)]


def _small_stage(n=40, d=6, N=16, L=2, t_bits=20, seed=0, dtype="u8", t=None):
    P = oracle.Params(N, oracle.rns_primes(N, L),
                      t if t is not None else oracle.plain_modulus(N, t_bits))
    g = np.random.default_rng(seed)
    if dtype == "u8":
        pts = g.integers(0, 256, (n, d)).astype(np.uint8)
        qv = g.integers(0, 256, d).astype(np.uint8)
    else:
        pts = g.integers(-127, 128, (n, d)).astype(np.int8)
        qv = g.integers(-127, 128, d).astype(np.int8)
    s = synthdata.gen_secret(N, seed + 1)
    a = synthdata.gen_uniform_a(P.qs, N, d, seed + 2)
    e = synthdata.gen_cbd_error(N, d, seed + 3)
    ct = oracle.encrypt_constants(P, s, a, e, [int(x) for x in qv])
    slot = synthdata.gen_slot_map(n, N, seed + 4)
    key = synthdata.gen_mask_key(seed + 5)
    return P, pts, qv, s, ct, slot, key


@pytest.mark.parametrize("dtype,t", [("u8", None), ("i8", None), ("u8", 1 << 20),
                                     ("i8", 1 << 19)])
def test_share_sum_is_squared_distance(dtype, t):
    """[client + server]_t = ||q - p||^2 for every real slot (closed form),
    with t the prime of the workloads or a power of two (the paper's choice,
    Section 5: the packing never needs slots of Z_t[x], so any t above the
    largest distance works),
    padding slots decrypt to their mask only, and the noise obeys the bound
    d N eta max|g| + (q mod t)(d max|g| + 2): the product's integer message
    W = sum_i [q_i]_t g_i + [P - r]_t is W = M + tK with |K| <= d max|g| + 2,
    and Delta t K = -(q mod t) K mod q."""
    P, pts, qv, s, ct, slot, key = _small_stage(dtype=dtype, t=t)
    n, d = pts.shape
    C = len(slot) // P.N
    qn2 = int((qv.astype(np.int64) ** 2).sum()) % P.t
    maxg = 2 * int(np.abs(pts.astype(np.int64)).max())
    bound = d * P.N * 21 * maxg + (P.q % P.t) * (d * maxg + 2)
    dist = ((pts.astype(np.int64) - qv.astype(np.int64)) ** 2).sum(axis=1)
    for k in range(C):
        g, nrm = oracle.chunk_plaintexts(pts, slot, P.N, k)
        out, r = oracle.server_chunk(P, ct, g, nrm, key, 77, k)
        cs = oracle.client_shares(P, out, s, qn2)
        ids = slot[k * P.N:(k + 1) * P.N]
        for j in range(P.N):
            tot = (int(cs[j]) + int(r[j])) % P.t
            if ids[j] >= 0:
                assert tot == dist[ids[j]]
            else:
                assert tot == qn2
        # noise of the product ciphertext against the message [V + P - r]_t
        V = [(-2 * int(pts[i].astype(np.int64) @ qv.astype(np.int64))
              if i >= 0 else 0) for i in ids]
        msg = [(V[j] + int(nrm[j]) - int(r[j])) % P.t for j in range(P.N)]
        v = oracle.noise(P, out, s, msg)
        assert max(abs(x) for x in v) <= bound < P.delta // 2
        # sampled coefficients agree with the full chunk
        js = [0, 3, P.N - 1]
        sc, sr = oracle.server_coeffs(P, ct, g, nrm, key, 77, k, js)
        assert (sc == out[:, :, js]).all() and (sr == r[js]).all()


def test_server_plaintext_lift_is_signed():
    """The plaintext of a point is -2p as a signed integer (not its Z_t
    representative): with a zero secret and zero error, c0 of the product is
    exactly Delta * sum_i m_i (-2 p_i) + Delta [||p||^2 - r]_t mod q_l."""
    P, pts, qv, s, ct, slot, key = _small_stage(n=16, d=3)
    zero_s = np.zeros(P.N, dtype=np.int8)
    a = np.zeros((3, P.L, P.N), dtype=np.uint64)
    e = np.zeros((3, P.N), dtype=np.int16)
    ct0 = oracle.encrypt_constants(P, zero_s, a, e, [int(x) for x in qv])
    g, nrm = oracle.chunk_plaintexts(pts, slot, P.N, 0)
    out, r = oracle.server_chunk(P, ct0, g, nrm, key, 1, 0)
    for j in range(P.N):
        pid = slot[j]
        V = -2 * int(pts[pid].astype(np.int64) @ qv.astype(np.int64))
        M = (int(nrm[j]) - int(r[j])) % P.t
        for l, ql in enumerate(P.qs):
            assert int(out[0, l, j]) == (P.delta * V + P.delta * M) % ql
            assert int(out[1, l, j]) == 0


# ---------------------------------------------------------------- top-k

def test_naive_topk_matches_sort():
    """Algorithm 1 returns the k smallest values in sorted order.  With
    distinct values the (value, ID) list is unique and equals a sort; with
    ties only the values are unique, so the IDs are checked for validity."""
    g = np.random.default_rng(5)
    distinct = g.permutation(400).tolist()
    ids = list(range(400))
    for k in (1, 3, 10, 400):
        v, i = oracle.naive_topk(distinct, ids, k)
        assert list(zip(v, i)) == sorted(zip(distinct, ids))[:k]
    vals = g.integers(0, 50, 400).tolist()
    for k in (1, 3, 10, 400):
        v, i = oracle.naive_topk(vals, ids, k)
        assert v == sorted(vals)[:k]
        assert len(set(i)) == k and all(vals[x] == y for x, y in zip(i, v))


def test_approx_topk_special_cases():
    g = np.random.default_rng(6)
    vals = g.permutation(1000)
    ids = np.arange(1000)
    # l = n: every bin is one item -> exact top-k
    assert oracle.approx_topk(vals, ids, 10, 1000) == oracle.naive_topk(
        vals.tolist(), ids.tolist(), 10)
    # k = 1: the global minimum is always its bin's minimum
    for l in (1, 7, 100):
        assert oracle.approx_topk(vals, ids, 1, l)[0] == [0]
    with pytest.raises(ValueError):
        oracle.approx_topk(vals, ids, 11, 10)
    assert oracle.bin_bounds(10, 3) == [(0, 4), (4, 7), (7, 10)]


def _closed_forms(n, l, k):
    b = n // l
    e_hit = l * (1 - math.comb(n - b, k) / math.comb(n, k))
    p_exact = 1.0
    for j in range(k):
        p_exact *= (n - j * b) / (n - j)
    return e_hit, p_exact


def test_approx_topk_brute_force_n16():
    """n=16, l=4, k=2: enumerate every placement of the two smallest values."""
    n, l, k = 16, 4, 2
    hits, exact, cnt = 0, 0, 0
    for p0, p1 in itertools.permutations(range(n), 2):
        vals = np.full(n, 100)
        rest = iter(range(2, n))
        for j in range(n):
            vals[j] = 0 if j == p0 else 1 if j == p1 else next(rest) + 10
        v, _ = oracle.approx_topk(vals, np.arange(n), k, l)
        inter = len({0, 1} & set(v))
        hits += inter
        exact += inter == 2
        cnt += 1
    e_hit, p_exact = _closed_forms(n, l, k)
    assert hits / cnt == pytest.approx(1.8) == pytest.approx(e_hit)
    assert exact / cnt == pytest.approx(0.8) == pytest.approx(p_exact)


def test_approx_topk_monte_carlo_matches_closed_form():
    """Theorems 1-2 (proofs in the appendix): with distinct values a true
    top-k item is returned iff it is the minimum of its bin, so |I| is the
    number of bins that hold at least one of the top k:
    E|I| = l(1 - C(n-n/l,k)/C(n,k)), P(exact) = prod_j (n - j n/l)/(n - j)."""
    n, l, k, T = 1000, 100, 10, 4000
    g = np.random.default_rng(8)
    base = np.arange(n)
    hits = np.empty(T)
    exact = np.empty(T)
    for it in range(T):
        vals = g.permutation(base)
        v, _ = oracle.approx_topk(vals, base, k, l)
        inter = len(set(range(k)) & set(v))
        hits[it] = inter
        exact[it] = inter == k
    e_hit, p_exact = _closed_forms(n, l, k)
    se_h = hits.std() / math.sqrt(T)
    se_p = math.sqrt(p_exact * (1 - p_exact) / T)
    assert abs(hits.mean() - e_hit) < 4 * se_h + 1e-9
    assert abs(exact.mean() - p_exact) < 4 * se_p
    # the workload values quoted for l=100 / l=1000
    assert _closed_forms(10_000, 100, 10)[0] == pytest.approx(9.566, abs=1e-3)
    assert _closed_forms(10 ** 6, 1000, 10)[1] == pytest.approx(0.956, abs=1e-3)


def test_sqdist_matches_numpy():
    g = np.random.default_rng(9)
    pts = g.integers(-127, 128, (300, 96)).astype(np.int8)
    qv = g.integers(-127, 128, 96).astype(np.int8)
    want = ((pts.astype(np.int64) - qv.astype(np.int64)) ** 2).sum(axis=1)
    assert (oracle.sqdist(qv, pts) == want).all()


# ---------------------------------------------------------------- packing

def test_packing_matches_paper_communication():
    """d query ciphertexts up and ceil(n/N) result ciphertexts down, each
    2 N log2(q) bits at N = 2^13, log2 q = 180, lands within 10% of the
    communication the paper reports for its linear scan."""
    with open(os.path.join(GOLD, "paper_comm_linear_scan.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    N, logq = 8192, 180
    for name, n, d, mb in rows:
        n, d, mb = int(n), int(d), float(mb)
        cts = d + -(-n // N)
        ours = cts * 2 * N * logq / 8 / 1e6
        assert abs(ours - mb) / mb < 0.10, name


# ---------------------------------------------------------------- seeded client randomness

def test_seeded_secret_is_uniform_ternary():
    """(x mod 3) - 1 over 64-bit ChaCha20 words: each of -1, 0, 1 with
    probability 1/3 (bias below 2^-62), so the counts of 2^16 draws lie
    within 5 sigma of N/3; different seeds give different keys."""
    N = 1 << 16
    s = oracle.sample_secret(11, N)
    assert s.dtype == np.int8 and set(np.unique(s)) == {-1, 0, 1}
    sigma = math.sqrt(N * (1 / 3) * (2 / 3))
    for v in (-1, 0, 1):
        assert abs(int((s == v).sum()) - N / 3) < 5 * sigma, v
    assert (oracle.sample_secret(11, N) == s).all()
    assert (oracle.sample_secret(12, 4096) != s[:4096]).any()
    # consecutive coefficients come from one block and are not equal in a run
    assert (s[:-1] != s[1:]).mean() > 0.6


def test_seeded_encryption_randomness_distributions():
    """a uniform in [0, q_l) (128-bit integers mod q_l, bias below 2^-74):
    mean within 5 sigma of q/2 and 16 equal bins pass a chi-square test at
    the 0.1% level; e a centred binomial with eta = 21: |e| <= 21, mean 0
    and variance eta/2 = 10.5 within 5 sigma."""
    P = oracle.Params(4096, oracle.rns_primes(4096, 2), 65537)
    a, e = oracle.sample_encryption(P, 21, 2, 8)
    for l, q in enumerate(P.qs):
        x = a[:, :, l, :].astype(np.float64).ravel() / q
        assert (a[:, :, l, :] < q).all()
        n = x.size
        assert abs(x.mean() - 0.5) < 5 * math.sqrt(1 / (12 * n))
        counts = np.bincount(np.minimum((x * 16).astype(int), 15), minlength=16)
        chi2 = float(((counts - n / 16) ** 2 / (n / 16)).sum())
        assert chi2 < 37.7, chi2  # 99.9% quantile, 15 degrees of freedom
    v = e.astype(np.float64).ravel()
    assert np.abs(e).max() <= 21
    assert abs(v.mean()) < 5 * math.sqrt(10.5 / v.size)
    # variance of the sample variance: (mu4 - sigma^4) / n, mu4 = 3 s^4 - s^2 / 2
    s2 = 10.5
    sd = math.sqrt((3 * s2 ** 2 - s2 / 2 - s2 ** 2) / v.size)
    assert abs(v.var() - s2) < 5 * sd, v.var()
    # streams differ by query, coordinate and limb
    assert (a[0, 0, 0] != a[1, 0, 0]).any() and (a[0, 0, 0] != a[0, 1, 0]).any()
    assert (e[0, 0] != e[0, 1]).any()


def test_seeded_encryption_decrypts():
    """Encryption with seeded (s, a, e) decrypts to the message and its noise
    is exactly e (Section 2.3)."""
    P = oracle.Params(64, oracle.rns_primes(64, 2), 257)
    s = oracle.sample_secret(3, 64)
    a, e = oracle.sample_encryption(P, 4, 1, 3)
    msgs = [5, 256, 100]
    ct = oracle.encrypt_constants(P, s, a[0], e[0], msgs)
    for i, m in enumerate(msgs):
        want = [m % P.t] + [0] * 63
        assert oracle.decrypt(P, ct[i], s) == want
        assert oracle.noise(P, ct[i], s, want) == [int(x) for x in e[0, i]]


# ---------------------------------------------------------------- circuit privacy

def _int_negacyclic(a, b):
    """Integer (unreduced) negacyclic product of two small polynomials."""
    N = len(a)
    out = [0] * N
    for u in range(N):
        for v in range(N):
            w = int(a[u]) * int(b[v])
            if u + v < N:
                out[u + v] += w
            else:
                out[u + v - N] -= w
    return out


def test_rerandomized_output_noise_decomposes_exactly():
    """Re-randomisation adds exactly the noise of a fresh encryption of zero
    plus the flood: noise(f') - noise(f) = e_pk u + e1 + e2 s + flood, term by
    term (integer polynomial products computed independently here), and the
    message is unchanged (client + server shares still equal the squared
    distances)."""
    P, pts, qv, s, ct, slot, key = _small_stage(n=30, d=5, N=16, L=2, t_bits=20)
    b = oracle.flood_bits(P)
    apk = synthdata.gen_uniform_a(P.qs, P.N, 1, 90)[0]
    epk = synthdata.gen_cbd_error(P.N, 1, 90)[0]
    pk = oracle.public_key(P, s, apk, epk)
    qn2 = int((qv.astype(np.int64) ** 2).sum()) % P.t
    dist = ((pts.astype(np.int64) - qv.astype(np.int64)) ** 2).sum(axis=1)
    for k in range(len(slot) // P.N):
        g, nrm = oracle.chunk_plaintexts(pts, slot, P.N, k)
        f, r = oracle.server_chunk(P, ct, g, nrm, key, 41, k)
        f2 = oracle.rerandomize(P, f, pk, key, 41, k, b)
        assert (f2[1] != f[1]).any()
        msg = oracle.decrypt(P, f, s)
        assert oracle.decrypt(P, f2, s) == msg
        u, e1, e2, flood = oracle.cp_randomness(P, key, 41, k, b)
        eu = _int_negacyclic(epk, u)
        e2s = _int_negacyclic(e2, s)
        want = [eu[j] + int(e1[j]) + e2s[j] + flood[j] for j in range(P.N)]
        got = [x - y for x, y in zip(oracle.noise(P, f2, s, msg), oracle.noise(P, f, s, msg))]
        assert got == want
        cs = oracle.client_shares(P, f2, s, qn2)
        ids = slot[k * P.N:(k + 1) * P.N]
        for j in range(P.N):
            tot = (int(cs[j]) + int(r[j])) % P.t
            assert tot == (dist[ids[j]] if ids[j] >= 0 else qn2)


def test_flood_width_and_margin():
    """The flood is uniform in [-2^b, 2^b) with 2^b <= Delta / 4; at the
    workloads' parameters the remaining margin holds the product noise bound
    d N eta max|g| + (q mod t)(d max|g| + 2) plus the re-randomisation noise
    (2 N eta + eta) with room to spare; flooding two bits wider would exceed
    the decryption margin Delta / 2 - t (a plausible off-by-two fails)."""
    for w, maxp in ((synthdata.WORKLOADS[1], 255), (synthdata.WORKLOADS[2], 255),
                    (synthdata.WORKLOADS[3], 127)):
        P = oracle.Params.for_workload(w.N, w.L, w.t_bits)
        b = oracle.flood_bits(P)
        assert (1 << b) <= P.delta // 4 < (1 << (b + 1))
        maxg = 2 * maxp
        prod = w.d * P.N * 21 * maxg + (P.q % P.t) * (w.d * maxg + 2)
        rr = 2 * P.N * 21 + 21
        assert (1 << b) + prod + rr < P.delta // 2 - P.t
        assert (1 << (b + 2)) > P.delta // 2
        # statistical distance of flood + v from flood, per ciphertext (N
        # coefficients): N (prod + rr) / 2^b; the bits it leaves
        # bound on the statistical distance: about 2^-82 at the N = 8192,
        # 162-bit workloads, only 2^-29 at the N = 4096, 108-bit one (the
        # paper's 108 bits need its 180-bit q)
        lam = b - math.log2(P.N * (prod + rr))
        assert lam > (80 if w.N == 8192 else 25), (w.cid, lam)
    P = oracle.Params(16, oracle.rns_primes(16, 2), 257)
    b = oracle.flood_bits(P)
    fl = []
    for ch in range(64):
        fl += oracle.cp_randomness(P, bytes(range(32)), 3, ch, b)[3]
    assert min(fl) >= -(1 << b) and max(fl) < (1 << b)
    x = np.array([f / (1 << b) for f in fl])
    assert abs(x.mean()) < 5 * math.sqrt(1 / (3 * len(x)))
    assert x.min() < -0.9 and x.max() > 0.9


def test_flooding_too_wide_breaks_decryption():
    """A flood of width 2^(b+3) (beyond the margin) decrypts wrongly somewhere:
    the margin check above is not vacuous."""
    P, pts, qv, s, ct, slot, key = _small_stage(n=16, d=3, N=16, L=2, t_bits=20)
    b = oracle.flood_bits(P)
    apk = synthdata.gen_uniform_a(P.qs, P.N, 1, 91)[0]
    epk = synthdata.gen_cbd_error(P.N, 1, 91)[0]
    pk = oracle.public_key(P, s, apk, epk)
    g, nrm = oracle.chunk_plaintexts(pts, slot, P.N, 0)
    f, r = oracle.server_chunk(P, ct, g, nrm, key, 5, 0)
    bad = sum(oracle.decrypt(P, oracle.rerandomize(P, f, pk, key, 5, k, b + 3), s)
              != oracle.decrypt(P, f, s) for k in range(4))
    assert bad >= 1


# ---------------------------------------------------------------- secret-shared points

def test_distances_on_secret_shared_points():
    """Points and norms held as additive shares p = p_c + p_s (mod t)
    (Section 4.2, last paragraph): the server's stage on its shares (full-range
    plaintexts) plus the client's cleartext terms -2 <q, p_c> + ||p||^2_c give
    [client + server]_t = ||q - p||^2 at every slot; the noise of the
    full-range product obeys d N eta max|g| + (q mod t)(d max|g| + 2) < Delta/2
    with max|g| = t / 2, and also at the workloads' parameters."""
    P, pts, qv, s, ct, slot, key = _small_stage(n=40, d=5, N=16, L=2, t_bits=20)
    g0 = np.random.default_rng(12)
    n, d = pts.shape
    pc = g0.integers(0, P.t, (n, d)).astype(np.int64)
    psh = (pts.astype(np.int64) - pc) % P.t
    nrm = (pts.astype(np.int64) ** 2).sum(axis=1)
    nc = g0.integers(0, P.t, n).astype(np.int64)
    nsh = (nrm - nc) % P.t
    q64 = qv.astype(np.int64)
    qn2 = int((q64 ** 2).sum()) % P.t
    bound = d * P.N * 21 * (P.t // 2) + (P.q % P.t) * (d * (P.t // 2) + 2)
    assert bound < P.delta // 2
    for k in range(len(slot) // P.N):
        g, nr = oracle.chunk_plaintexts_shares(psh, nsh, slot, P.N, k, P.t)
        assert np.abs(g).max() <= P.t // 2
        out, r = oracle.server_chunk(P, ct, g, nr, key, 9, k)
        dec = oracle.decrypt(P, out, s)
        ids = slot[k * P.N:(k + 1) * P.N]
        V = [(-2 * int(psh[i] @ q64) + int(nsh[i]) if i >= 0 else 0) for i in ids]
        msg = [(V[j] - int(r[j])) % P.t for j in range(P.N)]
        assert dec == msg
        assert max(abs(x) for x in oracle.noise(P, out, s, msg)) <= bound
        for j, i in enumerate(ids):
            if i < 0:
                continue
            client = (dec[j] + qn2 - 2 * int(pc[i] @ q64) + int(nc[i])) % P.t
            assert (client + int(r[j])) % P.t == int(((pts[i].astype(np.int64) - q64) ** 2).sum())
    for w in (synthdata.WORKLOADS[2], synthdata.WORKLOADS[3]):
        Pw = oracle.Params.for_workload(w.N, w.L, w.t_bits)
        bw = w.d * Pw.N * 21 * (Pw.t // 2) + (Pw.q % Pw.t) * (w.d * (Pw.t // 2) + 2)
        assert bw < Pw.delta // 2 - Pw.t
