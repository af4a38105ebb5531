// Negacyclic number-theoretic transform over Z_q[x]/(x^N + 1) for one
// polynomial per workgroup, N = 16 T residues held 16 per thread.
//
// Forward: merged-psi Cooley-Tukey (bit-reversed output), the butterfly at
// stride 2^p between indices j and j + 2^p uses Psi_rev[(N + j) >> (p + 1)],
// Psi_rev[m] = psi^bitrev(m) with psi a primitive 2N-th root of unity mod q.
// Inverse: Gentleman-Sande with Psi^-1 tables, then multiplication by N^-1.
// Lazy reduction (Harvey): forward values stay in [0, 4q), inverse in [0, 2q).
//
// Stages are grouped in passes of up to four index bits.  In a pass that
// covers bits [lo, lo + B) a thread holds the 16 residues whose index has
// its thread id (and, when B < 4, 4 - B extra bits from the register slot)
// in the other bit positions; the B stages of the pass run in registers and
// passes exchange data through LDS, padded by one word per 16 so that the
// strided patterns do not collide on banks.
#pragma once
#include "modarith.h"

namespace sanns {

__device__ __forceinline__ int lds_pad(int idx) { return idx + (idx >> 4); }

// Index of register slot a (0..15) of thread tid in a pass covering bits
// [lo, lo + B) of a 2^logN-point transform.
template <int B>
__device__ __forceinline__ int elem_index(int tid, int a, int lo, int logN) {
  const int r = (B == 4) ? tid : (tid | ((a >> B) << (logN - 4)));
  const int pb = a & ((1 << B) - 1);
  return (r & ((1 << lo) - 1)) | (pb << lo) | ((r >> lo) << (lo + B));
}

template <int B>
__device__ __forceinline__ void fwd_pass(uint64_t (&v)[16], int lo, int logN, int tid,
                                         const uint64_t* __restrict__ tw,
                                         const uint64_t* __restrict__ twp, uint64_t q) {
  const uint64_t q2 = 2 * q;
  const int N = 1 << logN;
#pragma unroll
  for (int rp = B - 1; rp >= 0; --rp) {
    const int p = lo + rp;
#pragma unroll
    for (int e = 0; e < (16 >> B); ++e) {
#pragma unroll
      for (int g = 0; g < (1 << (B - 1 - rp)); ++g) {
        const int a0 = (e << B) | (g << (rp + 1));
        const int w = (N + elem_index<B>(tid, a0, lo, logN)) >> (p + 1);
        const uint64_t W = tw[w], Wp = twp[w];
#pragma unroll
        for (int l = 0; l < (1 << rp); ++l) {
          const int a = a0 | l, b = a | (1 << rp);
          uint64_t X = v[a];
          X = X >= q2 ? X - q2 : X;
          const uint64_t T = shoup_lazy(v[b], W, Wp, q);
          v[a] = X + T;
          v[b] = X - T + q2;
        }
      }
    }
  }
}

template <int B>
__device__ __forceinline__ void inv_pass(uint64_t (&v)[16], int lo, int logN, int tid,
                                         const uint64_t* __restrict__ tw,
                                         const uint64_t* __restrict__ twp, uint64_t q) {
  const uint64_t q2 = 2 * q;
  const int N = 1 << logN;
#pragma unroll
  for (int rp = 0; rp < B; ++rp) {
    const int p = lo + rp;
#pragma unroll
    for (int e = 0; e < (16 >> B); ++e) {
#pragma unroll
      for (int g = 0; g < (1 << (B - 1 - rp)); ++g) {
        const int a0 = (e << B) | (g << (rp + 1));
        const int w = (N + elem_index<B>(tid, a0, lo, logN)) >> (p + 1);
        const uint64_t W = tw[w], Wp = twp[w];
#pragma unroll
        for (int l = 0; l < (1 << rp); ++l) {
          const int a = a0 | l, b = a | (1 << rp);
          const uint64_t X = v[a], Y = v[b];
          uint64_t s = X + Y;
          s = s >= q2 ? s - q2 : s;
          v[a] = s;
          v[b] = shoup_lazy(X - Y + q2, W, Wp, q);
        }
      }
    }
  }
}

template <int B>
__device__ __forceinline__ void lds_store(const uint64_t (&v)[16], uint64_t* lds, int lo,
                                          int logN, int tid) {
#pragma unroll
  for (int a = 0; a < 16; ++a) lds[lds_pad(elem_index<B>(tid, a, lo, logN))] = v[a];
}

template <int B>
__device__ __forceinline__ void lds_load(uint64_t (&v)[16], const uint64_t* lds, int lo,
                                         int logN, int tid) {
#pragma unroll
  for (int a = 0; a < 16; ++a) v[a] = lds[lds_pad(elem_index<B>(tid, a, lo, logN))];
}

// Geometry of pass j.  Forward passes walk the bits from the top, inverse
// passes from the bottom; only the last pass of either may be narrower.
__device__ __forceinline__ void fwd_geom(int j, int logN, int& lo, int& b) {
  const int hi = logN - 4 * j;
  lo = hi - 4 < 0 ? 0 : hi - 4;
  b = hi - lo;
}
__device__ __forceinline__ void inv_geom(int j, int logN, int& lo, int& b) {
  lo = 4 * j;
  b = logN - lo < 4 ? logN - lo : 4;
}
__device__ __forceinline__ int n_passes(int logN) { return (logN + 3) >> 2; }

// Global-memory index of register slot a for the first or last pass.
__device__ __forceinline__ int fwd_first_index(int tid, int a, int logN) {
  return elem_index<4>(tid, a, logN - 4, logN);
}
__device__ __forceinline__ int fwd_last_index(int tid, int a, int logN) {
  int lo, b;
  fwd_geom(n_passes(logN) - 1, logN, lo, b);
  switch (b) {
    case 1: return elem_index<1>(tid, a, lo, logN);
    case 2: return elem_index<2>(tid, a, lo, logN);
    case 3: return elem_index<3>(tid, a, lo, logN);
    default: return elem_index<4>(tid, a, lo, logN);
  }
}
__device__ __forceinline__ int inv_first_index(int tid, int a, int logN) {
  return elem_index<4>(tid, a, 0, logN);
}
__device__ __forceinline__ int inv_last_index(int tid, int a, int logN) {
  int lo, b;
  inv_geom(n_passes(logN) - 1, logN, lo, b);
  switch (b) {
    case 1: return elem_index<1>(tid, a, lo, logN);
    case 2: return elem_index<2>(tid, a, lo, logN);
    case 3: return elem_index<3>(tid, a, lo, logN);
    default: return elem_index<4>(tid, a, lo, logN);
  }
}

// Forward transform of the residues in v (loaded with fwd_first_index);
// returns them in [0, 4q) at fwd_last_index positions.  lds must hold
// lds_pad(N) + 1 words; the caller synchronises before reusing it.
__device__ __forceinline__ void ntt_fwd(uint64_t (&v)[16], uint64_t* lds, int logN, int tid,
                                        const uint64_t* __restrict__ tw,
                                        const uint64_t* __restrict__ twp, uint64_t q) {
  const int P = n_passes(logN);
  for (int j = 0; j < P; ++j) {
    int lo, b;
    fwd_geom(j, logN, lo, b);
    if (j > 0) {
      __syncthreads();
      switch (b) {
        case 1: lds_load<1>(v, lds, lo, logN, tid); break;
        case 2: lds_load<2>(v, lds, lo, logN, tid); break;
        case 3: lds_load<3>(v, lds, lo, logN, tid); break;
        default: lds_load<4>(v, lds, lo, logN, tid);
      }
    }
    switch (b) {
      case 1: fwd_pass<1>(v, lo, logN, tid, tw, twp, q); break;
      case 2: fwd_pass<2>(v, lo, logN, tid, tw, twp, q); break;
      case 3: fwd_pass<3>(v, lo, logN, tid, tw, twp, q); break;
      default: fwd_pass<4>(v, lo, logN, tid, tw, twp, q);
    }
    if (j + 1 < P) {
      // Only the last pass may be narrower than four bits.  Within a pass a
      // thread stores exactly the positions it loaded, so the one barrier
      // needed before the first store guards LDS still being read by a
      // previous transform of the same workgroup.
      if (j == 0) __syncthreads();
      lds_store<4>(v, lds, lo, logN, tid);
    }
  }
}

// Inverse transform (input at inv_first_index in [0, 2q), output at
// inv_last_index in [0, 2q), not yet multiplied by N^-1).
__device__ __forceinline__ void ntt_inv(uint64_t (&v)[16], uint64_t* lds, int logN, int tid,
                                        const uint64_t* __restrict__ tw,
                                        const uint64_t* __restrict__ twp, uint64_t q) {
  const int P = n_passes(logN);
  for (int j = 0; j < P; ++j) {
    int lo, b;
    inv_geom(j, logN, lo, b);
    if (j > 0) {
      __syncthreads();
      switch (b) {
        case 1: lds_load<1>(v, lds, lo, logN, tid); break;
        case 2: lds_load<2>(v, lds, lo, logN, tid); break;
        case 3: lds_load<3>(v, lds, lo, logN, tid); break;
        default: lds_load<4>(v, lds, lo, logN, tid);
      }
    }
    switch (b) {
      case 1: inv_pass<1>(v, lo, logN, tid, tw, twp, q); break;
      case 2: inv_pass<2>(v, lo, logN, tid, tw, twp, q); break;
      case 3: inv_pass<3>(v, lo, logN, tid, tw, twp, q); break;
      default: inv_pass<4>(v, lo, logN, tid, tw, twp, q);
    }
    if (j + 1 < P) {
      if (j == 0) __syncthreads();
      lds_store<4>(v, lds, lo, logN, tid);
    }
  }
}

}  // namespace sanns
