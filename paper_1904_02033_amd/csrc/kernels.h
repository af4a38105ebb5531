// Kernel argument structures shared by the kernels and the host launchers.
#pragma once
#include <stdint.h>
#include "modarith.h"

namespace sanns {

constexpr int kMaxLimbs = 4;
constexpr int kMaxWords = 8;  // 32-bit words of q (<= 4 * 54 bits) plus carry room

struct PrimeSet {
  Prime p[kMaxLimbs];
};

// Constants of the exact CRT decode.  M_l = q / q_l as 32-bit words.
struct DecodeConst {
  uint32_t qw[kMaxWords];              // q
  uint32_t Mw[kMaxLimbs][kMaxWords];   // q / q_l
  uint64_t inv[kMaxLimbs];             // (q / q_l)^-1 mod q_l
  uint64_t invp[kMaxLimbs];
  uint64_t tq[kMaxLimbs];              // t mod q_l  (= t)
  uint64_t tqp[kMaxLimbs];             // Shoup companion of t w.r.t. q_l
  uint32_t t;
  int words;                           // words used by q and the sums
};

// Twiddle tables of one limb (pairs of value and Shoup companion): N forward
// pairs psi_rev, then N inverse stage pairs (entry 2^p + m = omega^-(m N /
// 2^(p+1)), entry 0 unused), then N final factors psi^-j N^-1.
struct TwSet {
  const u64x2* tw[kMaxLimbs];
};

// Constants of the exact fold of the int8 matrix-core digit sums of one limb:
// a sum V = g0 + g1 2^32 + h 2^64 of signed 64-bit parts is reduced as
// (g0 + offa) + [ (g1 + offa) 2^32 ] + [ (h + offb) 2^64 ]  (mod q), or, when
// q = 2^54 - delta with 0 < delta < 2^22, with 2^54 = delta (mod q) alone.
struct DigitConst {
  uint64_t w32, w32p;  // 2^32 mod q and its Shoup companion
  uint64_t w64, w64p;  // 2^64 mod q and its Shoup companion
  uint64_t offa;       // smallest multiple of q >= 2^53
  uint64_t offb;       // smallest multiple of q >= 2^57
  uint64_t nq;         // 2^64 - q
  uint64_t twoq;       // 2 q
  int32_t delta;       // 2^54 - q if that is in (0, 2^22), else 0
};

struct DigitSet {
  DigitConst c[kMaxLimbs];
};

struct MaskKey {
  uint32_t k[8];
};

// Flooding of the circuit-private form: width b (flood uniform in
// [-2^b, 2^b)) and 2^b mod q_l per limb.
struct CpConst {
  uint64_t twob[kMaxLimbs];
  int b;
};

// Arguments of the persistent whole-batch kernel.
struct PersistArgs {
  const uint64_t* ct_in;    // [Q][d][2][L][N] coefficient form
  uint64_t* qntt;           // workspace: query NTT form, 27-bit halves
  const uint2* db;          // [L][C][d][N] halves
  const uint32_t* norms;    // [C][N]
  const uint64_t* qids;     // [Q]
  const uint32_t* work;     // [M][2] (query, chunk) or null for all pairs
  const void* tiles;        // MacTile<TQT, TCT>[n_tiles] when work is set
  uint64_t* ct_out;         // [M][2][L][N]
  uint32_t* share;          // [M][N]
  uint32_t* ctrl;           // kCtrlWords control words
  uint32_t* err;            // sticky error word
  int Q, d, L, C, M, n_tiles;
  uint32_t t;
  uint64_t tone;
  MaskKey K;
};

// One tile of the multiply-accumulate schedule: QT queries x CT chunks; the
// output index of pair (a, b) is out[a][b], -1 when the pair is padding.
template <int QT, int CT>
struct MacTile {
  int32_t q[QT];
  int32_t k[CT];
  int32_t out[QT][CT];
};

}  // namespace sanns
