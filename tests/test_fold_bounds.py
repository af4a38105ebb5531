"""Bounds of the short reductions for primes q = 2^54 - delta (delta < 2^22),
checked on the CPU with exact integers and 64-bit two's complement wrap,
step for step as the device code takes them:

* the fold of the 13 int8-digit diagonal sums S_s of the matrix-core
  multiply-accumulate (V = sum_s 256^s S_s, |S_s| < 7 2^21 and 0 <= S_12 <=
  2^19 for d <= 128) into a value below 2^57 congruent to V;
* x mod 2^54 + (x >> 54) delta, one conditional subtraction, for x < 2^60
  (the sums transpose, values below 2^58; the last step of the query
  transform, values below 2^60);
* the Horner step of the circuit-private form's flood residues.

Extreme diagonals (every sum at +bound or -bound, alternating signs, the
largest top sum) and random ones, for every such prime of the ring degrees
and limb counts the library derives.  Host arithmetic only, no GPU."""
import random

import oracle

M64 = (1 << 64) - 1
B = 7 * (1 << 21)   # |S_s| bound, d <= 128 (7 digit pairs x 2^14 x 128)
B12 = 1 << 19       # S_12 = sum of x_6 y_6 with x_6, y_6 in [0, 64]


def _s64(x):
    x &= M64
    return x - (1 << 64) if x >> 63 else x


def _i32(x):
    x &= 0xFFFFFFFF
    return x - (1 << 32) if x >> 31 else x


def fold_short(S, q):
    delta = (1 << 54) - q

    def group(s, base):
        g = base
        for j, k in enumerate((1, 1 << 8, 1 << 16, 1 << 24)):
            assert -(1 << 31) <= S[s + j] < 1 << 31
            g = _s64(g + S[s + j] * k)
        return g

    h = _s64(group(8, 0) + ((S[12] & 0xFFFFFFFF) << 32))
    hh = _i32((h & M64) >> 22)
    assert hh == h >> 22                      # the 32-bit field is the exact shift
    hl = h & 0x3FFFFF
    z = _s64(group(4, 0) + delta * hh + (hl << 32))
    zh = _i32((z & M64) >> 24)
    assert zh == z >> 24
    zl = z & 0xFFFFFF
    r = _s64(group(0, 2 * q) + 4 * delta * zh + (zl << 32))
    assert 0 <= r < 1 << 57
    return r


def reduce_short(x, q):
    delta = (1 << 54) - q
    assert 0 <= x < 1 << 60
    r = (x & ((1 << 54) - 1)) + (x >> 54) * delta
    assert r < 2 * q
    return r - q if r >= q else r


def _short_primes():
    out = set()
    for N in (64, 1024, 4096, 8192, 16384, 32768):
        for q in oracle.rns_primes(N, 6):
            if 0 < (1 << 54) - q < 1 << 22:
                out.add(q)
    return sorted(out)


def _diagonals(rng, mode):
    S = []
    for s in range(13):
        lo, hi = (0, B12) if s == 12 else (-(B - 1), B - 1)
        if mode == 0:
            v = rng.randint(lo, hi)
        elif mode == 1:
            v = hi
        elif mode == 2:
            v = lo
        elif mode == 3:
            v = hi if s % 2 else lo
        else:
            v = lo if s % 2 else hi
        S.append(v)
    return S


def test_short_fold_is_congruent_and_below_2_57():
    primes = _short_primes()
    assert len(primes) >= 10
    for q in primes:
        rng = random.Random(q)
        for it in range(400):
            S = _diagonals(rng, it % 5)
            V = sum(v << (8 * s) for s, v in enumerate(S))
            assert fold_short(S, q) % q == V % q, (q, S)


def test_short_reduction_below_2_60():
    for q in _short_primes():
        rng = random.Random(q + 1)
        xs = [0, 1, q - 1, q, 2 * q - 1, (1 << 54) - 1, 1 << 54, (1 << 58) - 1,
              (1 << 60) - 1] + [rng.randrange(1 << 60) for _ in range(2000)]
        for x in xs:
            assert reduce_short(x, q) == x % q, (q, x)


def test_short_horner_step():
    """The flood's Horner step r -> r 2^32 + w (mod q) of the circuit-private
    form: (r >> 22) delta + (r mod 2^22) 2^32 + w < 2^56, then the short
    reduction."""
    for q in _short_primes():
        delta = (1 << 54) - q
        rng = random.Random(q + 2)
        cases = [(0, 0), (q - 1, (1 << 32) - 1), (q - 1, 0), ((1 << 22) - 1, 1)]
        cases += [(rng.randrange(q), rng.randrange(1 << 32)) for _ in range(2000)]
        for r, w in cases:
            assert (r >> 22) < 1 << 32
            y = (r >> 22) * delta + ((r & 0x3FFFFF) << 32) + w
            assert y < 1 << 56
            assert reduce_short(y, q) == (r * (1 << 32) + w) % q, (q, r, w)


def test_workload_primes_take_the_short_forms():
    """The primes of every workload here (N = 4096 ... 16384, L <= 3) are
    2^54 - delta with delta < 2^22, so the batched schedules run the short
    forms; 50- and 52-bit primes do not."""
    for N in (4096, 8192, 16384):
        for q in oracle.rns_primes(N, 3):
            assert 0 < (1 << 54) - q < 1 << 22, (N, q)
    for bits in (50, 52):
        q = oracle.rns_primes(4096, 1, bits=bits)[0]
        assert (1 << 54) - q >= 1 << 22
