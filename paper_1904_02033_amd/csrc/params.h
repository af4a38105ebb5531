// Host-side parameter derivation: primes, roots of unity, twiddle tables and
// the per-limb constants of the kernels.
#pragma once
#include <stdint.h>
#include <string>
#include <vector>
#include "kernels.h"

namespace sanns {
namespace host {

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q);
uint64_t powmod(uint64_t a, uint64_t e, uint64_t q);
bool is_prime(uint64_t n);
uint64_t shoup_companion(uint64_t w, uint64_t q);  // floor(w 2^64 / q)

// The L largest primes below 2^bits with q = 1 mod 2N (descending).
std::vector<uint64_t> rns_primes(uint32_t N, uint32_t L, int bits = 54);
// Smallest prime >= 2^(bits-1) with t = 1 mod 2N.
uint64_t plain_modulus(uint32_t N, uint32_t bits);
// Smallest primitive 2N-th root of unity mod q.
uint64_t min_primitive_root_2n(uint32_t N, uint64_t q);

// Twiddles of one prime: [4][N] = psi_rev, psi_rev', ipsi_rev, ipsi_rev'.
std::vector<uint64_t> twiddle_table(uint32_t N, uint64_t q, uint64_t psi);

Prime prime_consts(uint32_t N, uint64_t q, uint64_t delta_mod_q);
DigitConst digit_consts(uint64_t q);

// Delta = floor(Q / t) mod q_l for every limb, Q = prod q_l.
std::vector<uint64_t> delta_mod_limbs(const std::vector<uint64_t>& qs, uint64_t t);

DecodeConst decode_consts(const std::vector<uint64_t>& qs, uint64_t t);

// Bit length of Delta = floor(prod q_l / t), t < 2^31.
int delta_bits(const std::vector<uint64_t>& qs, uint64_t t);
// 2^e mod q.
uint64_t pow2_mod(int e, uint64_t q);

// log2 of prod q_l, rounded up to whole bits.
int log2q_bits(const std::vector<uint64_t>& qs);

}  // namespace host
}  // namespace sanns
