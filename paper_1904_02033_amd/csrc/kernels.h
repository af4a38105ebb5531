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

// Twiddle tables of one limb: N (psi_rev, psi_rev') pairs, then N
// (ipsi_rev, ipsi_rev') pairs whose entry 0 holds ipsi_rev[1] N^-1.
struct TwSet {
  const u64x2* tw[kMaxLimbs];
};

struct MaskKey {
  uint32_t k[8];
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
