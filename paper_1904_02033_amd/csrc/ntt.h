// Negacyclic number-theoretic transform over Z_q[x]/(x^N + 1) for one
// polynomial per workgroup, N = 16 T residues held 16 per thread, with the
// transform size a compile-time parameter so that every index below folds
// to a per-thread base plus a constant.
//
// Forward: merged-psi Cooley-Tukey (bit-reversed output), the butterfly at
// stride 2^p between indices j and j + 2^p uses Psi_rev[(N + j) >> (p + 1)],
// Psi_rev[m] = psi^bitrev(m) with psi a primitive 2N-th root of unity mod q.
// The forward output at position k is the cyclic transform of (psi^j a_j) at
// frequency bitrev(k), so the inverse is a decimation-in-time Cooley-Tukey
// transform of that bit-reversed input with omega^-1 = psi^-2 (natural-order
// output), followed by the factor psi^-j N^-1 per coefficient: the butterfly
// at stride 2^p uses W_inv[2^p + (j mod 2^p)] = omega^-((j mod 2^p) N / 2^(p+1))
// (stage 0 multiplies by 1).
// Lazy reduction with the estimated Shoup quotient (products in [0, 4q) for
// any input below 2^63): no reduction inside either transform -- each
// butterfly maps values below B q to values below (B + 4) q (X + T and
// X + 4q - T; the inverse's twiddle-free stage 0 maps inputs below q to
// values below 3q), so after log2 N <= 14 stages they stay below 58 q < 2^60
// -- and one reduction at the end.
//
// Stages are grouped in passes of up to four index bits; the narrow pass (if
// log2 N is not a multiple of four) is the forward's first and the inverse's
// last, so both transforms meet at a pass over bits [0, 4).  In a pass over
// bits [lo, lo + B) a thread holds the 16 residues whose index has its thread
// id (and, when B < 4, 4 - B extra bits from the register slot) in the other
// bit positions; the B stages run in registers and passes exchange data
// through LDS (in two 32-bit halves), padded by one word per 16 against bank
// collisions.
//
// Global layouts that follow:
//   coefficient form: slot a of thread tid holds coefficient coef_index(tid, a),
//     consecutive threads reading consecutive words;
//   NTT form: slot a of thread tid holds the bit-reversed evaluation
//     a + 16 tid, stored at word ntt_slot(tid, a) = a T + tid, again
//     consecutive across threads.  Every consumer of NTT-form vectors works
//     slot-wise, so this storage order is private to the library.
#pragma once
#include "modarith.h"

namespace sanns {

template <int LOGN>
struct NttShape {
  static constexpr int N = 1 << LOGN;
  static constexpr int T = N >> 4;                 // threads per transform
  static constexpr int P = (LOGN + 3) >> 2;        // passes
  static constexpr int R = LOGN - 4 * (P - 1);     // bits of the narrow pass
  static constexpr int fwd_lo(int j) { return j == 0 ? LOGN - R : LOGN - R - 4 * j; }
  static constexpr int fwd_b(int j) { return j == 0 ? R : 4; }
  static constexpr int inv_lo(int j) { return 4 * j; }
  static constexpr int inv_b(int j) { return j == P - 1 ? R : 4; }
  // exchanges go through LDS in two 32-bit halves
  static constexpr size_t lds_bytes = (size_t)(N + (N >> 4)) * sizeof(uint32_t);
};

__device__ __forceinline__ constexpr int lds_pad(int idx) { return idx + (idx >> 4); }

// Index of register slot a (0..15) of thread tid in a pass over bits
// [LO, LO + B).  The thread's bits and the slot's bits land in disjoint
// positions, so eidx(tid, a) = eidx(tid, 0) + eidx(0, a), and the same holds
// after lds_pad or a right shift: addresses are a base plus a constant.
template <int LOGN, int B, int LO>
__device__ __forceinline__ constexpr int eidx(int tid, int a) {
  const int r = (B == 4) ? tid : (tid | ((a >> B) << (LOGN - 4)));
  const int pb = a & ((1 << B) - 1);
  return (r & ((1 << LO) - 1)) | (pb << LO) | ((r >> LO) << (LO + B));
}

template <int LOGN>
__device__ __forceinline__ int coef_index(int tid, int a) {
  using S = NttShape<LOGN>;
  return eidx<LOGN, S::R, LOGN - S::R>(tid, a);
}

template <int LOGN>
__device__ __forceinline__ int ntt_slot(int tid, int a) {
  return a * NttShape<LOGN>::T + tid;
}

// Twiddles of one stage (p1 = p + 1): (N + eidx(tid, a0)) >> p1 is
// ((N + eidx(tid, 0)) >> p1) + (eidx(0, a0) >> p1).  When every lane bit of
// the thread id sits below bit LO the base is the same across the wavefront.
template <int LOGN, int B, int LO>
__device__ __forceinline__ const u64x2* tw_stage(const u64x2* tw, int tid, int p1) {
  int b = (NttShape<LOGN>::N + eidx<LOGN, B, LO>(tid, 0)) >> p1;
  if (LO >= 6) b = __builtin_amdgcn_readfirstlane(b);
  return tw + b;
}

template <int LOGN, int B, int LO>
__device__ __forceinline__ void fwd_pass(uint64_t (&v)[16], int tid,
                                         const u64x2* __restrict__ tw, uint64_t q) {
  const uint64_t q4 = 4 * q, nq = 0 - q;
#pragma unroll
  for (int rp = B - 1; rp >= 0; --rp) {
    const int p = LO + rp;
    const u64x2* tb = tw_stage<LOGN, B, LO>(tw, tid, p + 1);
#pragma unroll
    for (int e = 0; e < (16 >> B); ++e) {
#pragma unroll
      for (int g = 0; g < (1 << (B - 1 - rp)); ++g) {
        const int a0 = (e << B) | (g << (rp + 1));
        const u64x2 W = tb[eidx<LOGN, B, LO>(0, a0) >> (p + 1)];
#pragma unroll
        for (int l = 0; l < (1 << rp); ++l) {
          const int a = a0 | l, b = a | (1 << rp);
          const uint64_t X = v[a];
          const uint64_t Tm = shoup_approx(v[b], W.x, W.y, nq);
          v[a] = X + Tm;
          v[b] = (X + q4) - Tm;
        }
      }
    }
  }
}

// Twiddle base of inverse stage p: index 2^p + (j mod 2^p), j = eidx(tid, x),
// is (2^p + (eidx(tid, 0) mod 2^p)) + (eidx(0, x) mod 2^p).  Only in the pass
// over the lowest bits does j mod 2^p not involve the thread id.
template <int LOGN, int B, int LO>
__device__ __forceinline__ const u64x2* tw_inv_stage(const u64x2* tw, int tid, int p) {
  int b = (1 << p) + (eidx<LOGN, B, LO>(tid, 0) & ((1 << p) - 1));
  if (LO == 0) b = __builtin_amdgcn_readfirstlane(b);
  return tw + b;
}

template <int LOGN, int B, int LO>
__device__ __forceinline__ void inv_pass(uint64_t (&v)[16], int tid,
                                         const u64x2* __restrict__ tw, uint64_t q) {
  const uint64_t q2 = 2 * q, q4 = 4 * q, nq = 0 - q;
#pragma unroll
  for (int rp = 0; rp < B; ++rp) {
    const int p = LO + rp;
    const u64x2* tb = tw_inv_stage<LOGN, B, LO>(tw, tid, p);
#pragma unroll
    for (int e = 0; e < (16 >> B); ++e) {
#pragma unroll
      for (int g = 0; g < (1 << (B - 1 - rp)); ++g) {
        const int a0 = (e << B) | (g << (rp + 1));
#pragma unroll
        for (int l = 0; l < (1 << rp); ++l) {
          const int a = a0 | l, b = a | (1 << rp);
          const uint64_t X = v[a], Y = v[b];
          if (p == 0) {
            // twiddle 1; inputs are below q
            v[a] = X + Y;
            v[b] = (X + q2) - Y;
          } else {
            const u64x2 W = tb[eidx<LOGN, B, LO>(0, a) & ((1 << p) - 1)];
            const uint64_t Tm = shoup_approx(Y, W.x, W.y, nq);
            v[a] = X + Tm;
            v[b] = (X + q4) - Tm;
          }
        }
      }
    }
  }
}

// Exchange between a pass over bits [LO0, LO0 + B0) and one over
// [LO1, LO1 + B1): every residue is written at its index and read back by the
// thread that holds that index in the next pass.  The words go through LDS
// as two 32-bit halves, so the buffer is N + N/16 32-bit words (a third
// workgroup of N/16 threads fits beside two others); the barrier between the
// halves keeps the high halves from overwriting low halves still being read.
// Each thread writes exactly the indices it read in the previous exchange, so
// no barrier is needed before the first store of the next exchange.
template <int LOGN, int B0, int LO0, int B1, int LO1>
__device__ __forceinline__ void lds_exchange(uint64_t (&v)[16], uint64_t* lds, int tid) {
  uint32_t* w = reinterpret_cast<uint32_t*>(lds);
  uint32_t* st = w + lds_pad(eidx<LOGN, B0, LO0>(tid, 0));
  const uint32_t* ld = w + lds_pad(eidx<LOGN, B1, LO1>(tid, 0));
  uint32_t lo[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) st[lds_pad(eidx<LOGN, B0, LO0>(0, a))] = (uint32_t)v[a];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 16; ++a) lo[a] = ld[lds_pad(eidx<LOGN, B1, LO1>(0, a))];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 16; ++a) st[lds_pad(eidx<LOGN, B0, LO0>(0, a))] = (uint32_t)(v[a] >> 32);
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 16; ++a)
    v[a] = lo[a] | ((uint64_t)ld[lds_pad(eidx<LOGN, B1, LO1>(0, a))] << 32);
}

template <int LOGN, int J>
__device__ __forceinline__ void fwd_from(uint64_t (&v)[16], uint64_t* lds, int tid,
                                         const u64x2* __restrict__ tw, uint64_t q) {
  using S = NttShape<LOGN>;
  constexpr int LO = S::fwd_lo(J), B = S::fwd_b(J);
  fwd_pass<LOGN, B, LO>(v, tid, tw, q);
  if constexpr (J + 1 < S::P) {
    // the barrier before the first store guards LDS still read by an
    // earlier transform of the workgroup
    if (J == 0) __syncthreads();
    lds_exchange<LOGN, B, LO, S::fwd_b(J + 1), S::fwd_lo(J + 1)>(v, lds, tid);
    fwd_from<LOGN, J + 1>(v, lds, tid, tw, q);
  }
}

template <int LOGN, int J>
__device__ __forceinline__ void inv_from(uint64_t (&v)[16], uint64_t* lds, int tid,
                                         const u64x2* __restrict__ tw, const Prime& P) {
  using S = NttShape<LOGN>;
  constexpr int LO = S::inv_lo(J), B = S::inv_b(J);
  inv_pass<LOGN, B, LO>(v, tid, tw, P.q);
  if constexpr (J + 1 < S::P) {
    if (J == 0) __syncthreads();
    lds_exchange<LOGN, B, LO, S::inv_b(J + 1), S::inv_lo(J + 1)>(v, lds, tid);
    inv_from<LOGN, J + 1>(v, lds, tid, tw, P);
  }
}

// Forward transform.  Input: residues below q, slot a = coefficient
// coef_index(tid, a).  Output: slot a = evaluation a + 16 tid in [0, q).
// lds holds NttShape<LOGN>::lds_bytes; the caller synchronises before reusing it.
// PM: q = 2^54 - delta with delta = pm_delta(q) != 0 (the last reduction by
// 2^54 = delta (mod q) instead of a Shoup product).
template <int LOGN, bool PM = false>
__device__ __forceinline__ void ntt_fwd(uint64_t (&v)[16], uint64_t* lds, int tid,
                                        const u64x2* __restrict__ tw, const Prime& P) {
  static_assert(LOGN <= 14, "forward values must stay below 2^60");
  fwd_from<LOGN, 0>(v, lds, tid, tw, P.q);
  const uint64_t nq = 0 - P.q;
  const uint32_t pd = pm_delta(P.q);
#pragma unroll
  for (int a = 0; a < 16; ++a)
    v[a] = PM ? reduce_pm60(v[a], pd, P.q)
              : csub(csub(shoup_approx(v[a], 1, P.one, nq), 2 * P.q), P.q);
}

// Inverse transform.  Input: residues below q, slot a = evaluation a + 16 tid
// (the forward's output order).  Output: slot a = coefficient
// coef_index(tid, a) in [0, q).  tw points at the limb's inverse stage table,
// which is followed by the N (psi^-j N^-1, companion) pairs of the final
// factor.
template <int LOGN>
__device__ __forceinline__ void ntt_inv(uint64_t (&v)[16], uint64_t* lds, int tid,
                                        const u64x2* __restrict__ tw, const Prime& P) {
  static_assert(LOGN <= 14, "inverse values must stay below 2^60");
  inv_from<LOGN, 0>(v, lds, tid, tw, P);
  const u64x2* F = tw + NttShape<LOGN>::N;
  const uint64_t nq = 0 - P.q;
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const u64x2 f = F[coef_index<LOGN>(tid, a)];
    v[a] = csub(csub(shoup_approx(v[a], f.x, f.y, nq), 2 * P.q), P.q);
  }
}

}  // namespace sanns
