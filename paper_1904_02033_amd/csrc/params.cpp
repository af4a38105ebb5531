// Host-side parameter derivation (primes, roots, twiddles, kernel constants).
#include "params.h"

#include <algorithm>
#include <cstring>
#include <stdexcept>

namespace sanns {
namespace host {

typedef unsigned __int128 u128;

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulmod(r, a, q);
    a = mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for 64-bit n (the first twelve prime bases
// suffice below 3.3e24).
bool is_prime(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

uint64_t shoup_companion(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

std::vector<uint64_t> rns_primes(uint32_t N, uint32_t L, int bits) {
  const uint64_t m = 2ull * N;
  uint64_t c = (((1ull << bits) - 1) / m) * m + 1;
  std::vector<uint64_t> out;
  while (out.size() < L && c > m) {
    if (is_prime(c)) out.push_back(c);
    c -= m;
  }
  return out;
}

uint64_t plain_modulus(uint32_t N, uint32_t bits) {
  const uint64_t m = 2ull * N;
  const uint64_t lo = 1ull << (bits - 1);
  uint64_t c = ((lo + m - 1) / m) * m + 1;
  while (!is_prime(c)) c += m;
  return c;
}

uint64_t min_primitive_root_2n(uint32_t N, uint64_t q) {
  const uint64_t two_n = 2ull * N;
  uint64_t root = 0;
  for (uint64_t g = 2; g < q; ++g) {
    const uint64_t c = powmod(g, (q - 1) / two_n, q);
    if (powmod(c, N, q) == q - 1) {
      root = c;
      break;
    }
  }
  if (!root) throw std::runtime_error("no primitive 2N-th root of unity");
  // every primitive 2N-th root is root^k for odd k; keep the smallest
  uint64_t best = root, cur = root;
  const uint64_t root2 = mulmod(root, root, q);
  for (uint64_t k = 3; k < two_n; k += 2) {
    cur = mulmod(cur, root2, q);
    best = std::min(best, cur);
  }
  return best;
}

static uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

std::vector<uint64_t> twiddle_table(uint32_t N, uint64_t q, uint64_t psi) {
  int logN = 0;
  while ((1u << logN) < N) ++logN;
  const uint64_t ipsi = powmod(psi, q - 2, q);
  const uint64_t iw = mulmod(ipsi, ipsi, q);  // omega^-1, omega = psi^2
  const uint64_t ninv = powmod(N % q, q - 2, q);
  std::vector<uint64_t> pw(N), iww(N);
  pw[0] = iww[0] = 1;
  for (uint32_t i = 1; i < N; ++i) {
    pw[i] = mulmod(pw[i - 1], psi, q);
    iww[i] = mulmod(iww[i - 1], iw, q);
  }
  // [0, 2N): forward (Psi_rev, companion) pairs;
  // [2N, 4N): inverse stage pairs, entry 2^p + m = omega^-(m N / 2^(p+1));
  // [4N, 6N): final factor psi^-j N^-1 pairs in coefficient order.
  std::vector<uint64_t> t(6 * (size_t)N, 0);
  for (uint32_t m = 0; m < N; ++m) {
    const uint32_t r = bitrev(m, logN);
    t[2 * (size_t)m] = pw[r];
    t[2 * (size_t)m + 1] = shoup_companion(pw[r], q);
  }
  for (int p = 0; p < logN; ++p)
    for (uint32_t m = 0; m < (1u << p); ++m) {
      const uint64_t w = iww[(size_t)m * (N >> (p + 1))];
      const size_t i = 2 * (size_t)N + 2 * ((1u << p) + m);
      t[i] = w;
      t[i + 1] = shoup_companion(w, q);
    }
  uint64_t f = ninv;
  for (uint32_t j = 0; j < N; ++j) {
    t[4 * (size_t)N + 2 * j] = f;
    t[4 * (size_t)N + 2 * j + 1] = shoup_companion(f, q);
    f = mulmod(f, ipsi, q);
  }
  return t;
}

Prime prime_consts(uint32_t N, uint64_t q, uint64_t delta_mod_q) {
  Prime P;
  P.q = q;
  P.one = (uint64_t)((((u128)1) << 64) / q);
  P.c54 = (uint64_t)((((u128)1) << 54) % q);
  P.c54p = shoup_companion(P.c54, q);
  P.delta = delta_mod_q;
  P.deltap = shoup_companion(delta_mod_q, q);
  P.ninv = powmod(N % q, q - 2, q);
  P.ninvp = shoup_companion(P.ninv, q);
  return P;
}

DigitConst digit_consts(uint64_t q) {
  DigitConst D;
  D.w32 = (uint64_t)((((u128)1) << 32) % q);
  D.w32p = shoup_companion(D.w32, q);
  D.w64 = (uint64_t)((((u128)1) << 64) % q);
  D.w64p = shoup_companion(D.w64, q);
  D.offa = (((1ull << 53) + q - 1) / q) * q;
  D.offb = (((1ull << 57) + q - 1) / q) * q;
  D.nq = 0 - q;
  D.twoq = 2 * q;
  D.delta = (int32_t)pm_delta(q);
  return D;
}

// floor(Q/t) = (Q - (Q mod t)) / t  and  Q = 0 mod q_l, so
// floor(Q/t) = -(Q mod t) t^-1  (mod q_l).
std::vector<uint64_t> delta_mod_limbs(const std::vector<uint64_t>& qs, uint64_t t) {
  uint64_t qmodt = 1 % t;
  for (uint64_t q : qs) qmodt = mulmod(qmodt, q % t, t);
  std::vector<uint64_t> out;
  for (uint64_t q : qs) {
    const uint64_t tinv = powmod(t % q, q - 2, q);
    const uint64_t v = mulmod(qmodt % q, tinv, q);
    out.push_back(v == 0 ? 0 : q - v);
  }
  return out;
}

// Little-endian 32-bit words of x * y (x as words, y < 2^64).
static std::vector<uint32_t> mw_mul(const std::vector<uint32_t>& x, uint64_t y) {
  std::vector<uint32_t> out(x.size() + 2, 0);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  for (int part = 0; part < 2; ++part) {
    const uint32_t yy = part ? y1 : y0;
    uint64_t carry = 0;
    for (size_t w = 0; w + part < out.size(); ++w) {
      const uint64_t xv = w < x.size() ? x[w] : 0;
      const u128 cur = (u128)out[w + part] + (u128)xv * yy + carry;
      out[w + part] = (uint32_t)cur;
      carry = (uint64_t)(cur >> 32);
    }
  }
  while (out.size() > 1 && out.back() == 0) out.pop_back();
  return out;
}

DecodeConst decode_consts(const std::vector<uint64_t>& qs, uint64_t t) {
  DecodeConst D;
  std::memset(&D, 0, sizeof D);
  const size_t L = qs.size();
  std::vector<uint32_t> qw = {1};
  for (uint64_t q : qs) qw = mw_mul(qw, q);
  if (qw.size() + 1 > (size_t)kMaxWords) throw std::runtime_error("modulus too wide");
  for (size_t w = 0; w < qw.size(); ++w) D.qw[w] = qw[w];
  D.words = (int)qw.size() + 1;
  for (size_t l = 0; l < L; ++l) {
    std::vector<uint32_t> M = {1};
    uint64_t Mmod = 1;
    for (size_t j = 0; j < L; ++j)
      if (j != l) {
        M = mw_mul(M, qs[j]);
        Mmod = mulmod(Mmod, qs[j] % qs[l], qs[l]);
      }
    for (size_t w = 0; w < M.size() && w < (size_t)kMaxWords; ++w) D.Mw[l][w] = M[w];
    D.inv[l] = powmod(Mmod, qs[l] - 2, qs[l]);
    D.invp[l] = shoup_companion(D.inv[l], qs[l]);
    D.tq[l] = t;
    D.tqp[l] = shoup_companion(t, qs[l]);
  }
  D.t = (uint32_t)t;
  return D;
}

int delta_bits(const std::vector<uint64_t>& qs, uint64_t t) {
  std::vector<uint32_t> qw = {1};
  for (uint64_t q : qs) qw = mw_mul(qw, q);
  // long division of the words by t < 2^31, most significant word first
  uint64_t rem = 0;
  std::vector<uint32_t> quo(qw.size(), 0);
  for (size_t i = qw.size(); i-- > 0;) {
    const uint64_t cur = (rem << 32) | qw[i];
    quo[i] = (uint32_t)(cur / t);
    rem = cur % t;
  }
  int bits = 0;
  for (size_t i = quo.size(); i-- > 0;)
    if (quo[i]) {
      bits = 32 * (int)i;
      for (uint32_t top = quo[i]; top; top >>= 1) ++bits;
      break;
    }
  return bits;
}

uint64_t pow2_mod(int e, uint64_t q) {
  uint64_t r = 1 % q;
  for (int i = 0; i < e; ++i) r = (uint64_t)(((u128)r << 1) % q);
  return r;
}

int log2q_bits(const std::vector<uint64_t>& qs) {
  std::vector<uint32_t> qw = {1};
  for (uint64_t q : qs) qw = mw_mul(qw, q);
  int bits = 32 * (int)(qw.size() - 1);
  uint32_t top = qw.back();
  while (top) {
    ++bits;
    top >>= 1;
  }
  // exact log2 is below `bits`; a power of two never occurs for a product
  // of odd primes
  return bits;
}

}  // namespace host
}  // namespace sanns
