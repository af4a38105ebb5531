// HIP kernels of the homomorphic distance stage (gfx950).
//
// Data layouts (all device memory):
//   ciphertexts        [.][2][L][N] uint64, coefficient form, residues < q_l
//   query NTT form     [Q][d][2][L][N] uint64 (bit-reversed NTT order)
//   database residues  [L][C][d][N] uint2: 27-bit halves of the NTT form
//   database norms     [C][N] uint32
//   server shares      [M][N] uint32
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "launch.h"
#include "ntt.h"
#include "chacha.h"

namespace sanns {

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------

// General product of two residues (Karatsuba on 27-bit halves, then the
// same fold as the multiply-accumulate).
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, const Prime& P) {
  uint32_t a0, a1, b0, b1;
  split27(a, a0, a1);
  split27(b, b0, b1);
  Acc3 acc;
  acc.lo = mul32x32(a0, b0);
  acc.hi = mul32x32(a1, b1);
  acc.mid = mul32x32(a0 + a1, b0 + b1);
  return acc3_reduce(acc, P);
}

// --------------------------------------------------------------------------
// forward / inverse transforms of independent polynomials
// --------------------------------------------------------------------------

// Forward transform of polynomial p (limb p % L) by one workgroup.  Output
// forms (split):
//   0  uint64 residues, polynomial-major like the input;
//   1  27-bit halves (uint2), polynomial-major: the form the 64-bit
//      multiply-accumulate kernels consume;
//   2  uint64 residues grouped by 32 slots, [L][R][N/32][d][32] with rows
//      r = 2q + c (R = 2Q) for polynomial p = ((q d + i) 2 + c) L + l: each
//      32-slot group of a row is one contiguous block over the coordinates,
//      the form the digit transpose of the matrix-core schedule reads.
template <int LOGN, int SPLIT, bool PM = false>
__device__ __forceinline__ void ntt_fwd_poly(int p, int tid, uint64_t* lds,
                                             const uint64_t* __restrict__ in,
                                             uint64_t* __restrict__ out, int L,
                                             const PrimeSet& ps, const TwSet& tws,
                                             uint32_t* err, int d = 0, int R = 0) {
  constexpr int N = NttShape<LOGN>::N;
  const int l = p % L;
  const Prime& P = ps.p[l];
  const uint64_t* src = in + (size_t)p * N;
  uint64_t v[16];
  bool bad = false;
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    v[a] = __builtin_nontemporal_load(src + coef_index<LOGN>(tid, a));  // read once
    bad |= v[a] >= P.q;
  }
  if (bad && err) atomicOr(err, 1u);
  ntt_fwd<LOGN, PM>(v, lds, tid, tws.tw[l], P);
  uint64_t* dst = out + (size_t)p * N;
  if constexpr (SPLIT == 2) {
    const int c = (p / L) & 1, i = (p / (2 * L)) % d, q = p / (2 * L * d);
    uint64_t* base = out + (((size_t)l * R + 2 * q + c) * (N / 32) * d + i) * 32;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int s = ntt_slot<LOGN>(tid, a);
      // read once, by the digit transpose
      __builtin_nontemporal_store(v[a], base + (size_t)(s >> 5) * d * 32 + (s & 31));
    }
  } else if constexpr (SPLIT == 1) {
    uint2* dst2 = reinterpret_cast<uint2*>(dst);
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      uint2 y;
      split27(v[a], y.x, y.y);
      dst2[ntt_slot<LOGN>(tid, a)] = y;
    }
  } else {
#pragma unroll
    for (int a = 0; a < 16; ++a) dst[ntt_slot<LOGN>(tid, a)] = v[a];
  }
}

// Waves per SIMD the transform kernels are compiled for: the largest of 4,
// 6 and 8 at which the compiler fits them in registers without spilling
// (checked for every log2 N).  The forward needs 64-72 registers; at eight
// waves (64 registers) the digit form fits except for log2 N = 8, 9 and 14,
// the other forms do not.  The inverse with the mask takes up to 128
// registers at four waves and 75-80 at six, where it spills for log2 N = 9,
// 11, 12 and 14 (9 spills at four waves too, so it keeps six).
constexpr int ntt_fwd_waves(int logn, int split) {
  return split == 2 && logn != 8 && logn != 9 && logn != 14 ? 8 : 6;
}
constexpr int intt_mask_waves(int logn) {
  return logn == 11 || logn == 12 || logn == 14 ? 4 : 6;
}

// One polynomial per workgroup (PM: every prime is 2^54 - delta, delta < 2^22).
template <int LOGN, int SPLIT, bool PM = false>
__global__ void __launch_bounds__(NttShape<LOGN>::T, ntt_fwd_waves(LOGN, SPLIT))
k_ntt_fwd(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, int L, PrimeSet ps,
          TwSet tws, uint32_t* err, int d, int R) {
  extern __shared__ uint64_t lds[];
  ntt_fwd_poly<LOGN, SPLIT, PM>(blockIdx.x, threadIdx.x, lds, in, out, L, ps, tws, err, d, R);
}

// In-place inverse transform, result multiplied by N^-1 and in [0, q).
template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T, 4)
k_ntt_inv(uint64_t* __restrict__ io, int L, PrimeSet ps, TwSet tws) {
  extern __shared__ uint64_t lds[];
  constexpr int N = NttShape<LOGN>::N;
  const int tid = threadIdx.x;
  const int p = blockIdx.x, l = p % L;
  const Prime& P = ps.p[l];
  uint64_t* buf = io + (size_t)p * N;
  uint64_t v[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) v[a] = buf[ntt_slot<LOGN>(tid, a)];
  ntt_inv<LOGN>(v, lds, tid, tws.tw[l] + N, P);
  __syncthreads();  // every thread has read its inputs before any overwrite
#pragma unroll
  for (int a = 0; a < 16; ++a) buf[coef_index<LOGN>(tid, a)] = v[a];
}

// --------------------------------------------------------------------------
// server masks (ChaCha20 in chacha.h), four slots per block
// --------------------------------------------------------------------------

__device__ __forceinline__ void work_pair(const uint32_t* work, int m, int C, int& qi, int& k) {
  if (work) {
    qi = (int)work[2 * m];
    k = (int)work[2 * m + 1];
  } else {
    qi = m / C;
    k = m % C;
  }
}

// Thread per (output m, block b).
__global__ void __launch_bounds__(256)
k_masks(MaskKey K, const uint64_t* __restrict__ qids, const uint32_t* __restrict__ work,
        int C, int M, int N, uint32_t t, uint64_t tone, uint32_t* __restrict__ share) {
  const int nb = N >> 2;
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)M * nb) return;
  const int m = (int)(g / nb), b = (int)(g % nb);
  int qi, k;
  work_pair(work, m, C, qi, k);
  mask_block(K, qids[qi], k, b, t, tone, share + (size_t)m * N);
}

// --------------------------------------------------------------------------
// inverse transform of the products plus the norm-and-mask plaintext
// --------------------------------------------------------------------------

// Polynomial p = (m 2 + c) L + l of ct_out: INTT, times N^-1, and for c = 0
// add Delta_l [norm - r]_t at every coefficient.
template <int LOGN>
__device__ __forceinline__ void intt_mask_poly(int p, int tid, uint64_t* lds,
                                               uint64_t* __restrict__ ct,
                                               const uint32_t* __restrict__ share,
                                               const uint32_t* __restrict__ norms,
                                               const uint32_t* __restrict__ work, int C, int L,
                                               uint32_t t, const PrimeSet& ps, const TwSet& tws) {
  constexpr int N = NttShape<LOGN>::N;
  const int l = p % L, c = (p / L) & 1, m = p / (2 * L);
  const Prime& P = ps.p[l];
  uint64_t* buf = ct + (size_t)p * N;
  uint64_t v[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) v[a] = __builtin_nontemporal_load(buf + ntt_slot<LOGN>(tid, a));
  ntt_inv<LOGN>(v, lds, tid, tws.tw[l] + N, P);
  if (c == 0) {
    int qi, k;
    work_pair(work, m, C, qi, k);
    const uint32_t* nrm = norms + (size_t)k * N;
    const uint32_t* r = share + (size_t)m * N;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int j = coef_index<LOGN>(tid, a);
      const uint32_t pn = nrm[j], rj = r[j];
      const uint64_t mv = pn >= rj ? pn - rj : pn + t - rj;
      v[a] = addmod(v[a], shoup(mv, P.delta, P.deltap, P.q), P.q);
    }
  }
  __syncthreads();  // every thread has read its inputs before any overwrite
#pragma unroll
  for (int a = 0; a < 16; ++a) __builtin_nontemporal_store(v[a], buf + coef_index<LOGN>(tid, a));
}

// The polynomial of ct_out that workgroup b of a grid of 8 ceil(n / 8) takes
// (n = 2 L M polynomials; -1 for the grid's padding).  Consecutive blocks go
// to the eight XCDs in turn, so block b is the (b / 8)-th of XCD b % 8, and
// each XCD takes a contiguous range of this order: for all pairs (Qa > 0
// queries, M = Qa C) chunk-major, the outputs of one chunk for every query
// back to back, so that the chunk's norms are fetched once into that XCD's
// L2; and the 2L polynomials of an output adjacent, so that the L that read
// its mask row find it there.  A work list (Qa = 0) keeps its own order.
__device__ __forceinline__ int intt_poly_of_block(int b, int n, int Qa, int C, int L) {
  const int per = (n + 7) >> 3;
  const int idx = (b & 7) * per + (b >> 3);
  if (idx >= n) return -1;
  if (Qa <= 0) return idx;
  const int l = idx % L, c = (idx / L) & 1, r = idx / (2 * L);
  return (((r % Qa) * C + r / Qa) * 2 + c) * L + l;
}

// At N = 8192: six waves per SIMD (78 registers, three workgroups of 512
// threads per CU) run 8% faster than four (126 registers, two workgroups).
template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T, intt_mask_waves(LOGN))
k_intt_mask(uint64_t* __restrict__ ct, const uint32_t* __restrict__ share,
            const uint32_t* __restrict__ norms, const uint32_t* __restrict__ work, int C,
            int L, uint32_t t, PrimeSet ps, TwSet tws, int n, int Qa) {
  extern __shared__ uint64_t lds[];
  const int p = intt_poly_of_block(blockIdx.x, n, Qa, C, L);
  if (p < 0) return;
  intt_mask_poly<LOGN>(p, threadIdx.x, lds, ct, share, norms, work, C, L, t, ps, tws);
}

// --------------------------------------------------------------------------
// circuit privacy: each output gets a fresh encryption of zero under its
// query's public key pk = (p0, p1),  (p0 u + e1 + flood, p1 u + e2),  with
// u ternary, e1 and e2 centred binomial (eta = 21) and the flood uniform in
// [-2^b, 2^b), all drawn from the server's mask key and the output's mask
// nonce (query id, chunk) at block counters s 2^24 + block for streams
// s = 1 (u), 2 (e1), 3 (e2), 4 (flood)
// --------------------------------------------------------------------------

constexpr uint32_t kCpStreamU = 1u << 24, kCpStreamE1 = 2u << 24, kCpStreamE2 = 3u << 24,
                   kCpStreamFlood = 4u << 24;

__device__ __forceinline__ uint64_t word64_of(const uint32_t (&o)[16], int n) {
  return (uint64_t)o[2 * n] | (uint64_t)o[2 * n + 1] << 32;
}

__device__ __forceinline__ int cbd21(uint64_t x) {
  return __popcll(x & 0x1FFFFFull) - __popcll((x >> 21) & 0x1FFFFFull);
}

__device__ __forceinline__ uint64_t lift_small(int x, uint64_t q) {
  return x < 0 ? q - (uint64_t)(-x) : (uint64_t)x;
}

// (X mod 2^(b+1)) - 2^b  mod q, X the 256-bit little-endian integer w[0..7]:
// Horner over the 32-bit words from the top kept word down.  r 2^32 is a
// Shoup product with 2^32 mod q (q > 2^32 keeps r + w below 2q), or, for q =
// 2^54 - delta with delta < 2^22, (r >> 22) delta + (r mod 2^22) 2^32 (as
// 2^54 = delta mod q; below 2^55 with r < 2^54), reduced with w added.
__device__ __forceinline__ uint64_t flood_residue(const uint32_t* w, int b, uint64_t twob,
                                                  const DigitConst& D, uint64_t q) {
  const int bits = b + 1;
  const uint32_t pd = pm_delta(q);
  uint64_t r = 0;
  for (int i = (bits - 1) >> 5; i >= 0; --i) {
    const int keep = bits - 32 * i;
    const uint32_t x = keep >= 32 ? w[i] : (w[i] & ((1u << keep) - 1u));
    if (pd) {
      r = reduce_pm60((uint64_t)(uint32_t)(r >> 22) * pd + ((r & 0x3fffffull) << 32) + x, pd, q);
    } else {
      r = shoup(r, D.w32, D.w32p, q) + x;
      if (r >= q) r -= q;
    }
  }
  return submod(r, twob, q);
}

// Workgroup per (output m, limb l): u in NTT form (generated cooperatively
// into LDS, then transformed), times the NTT form of the query's public key,
// added to both NTT-form components of ct_out.
template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T, 4)
k_rerand(MaskKey K, const uint64_t* __restrict__ qids, const uint32_t* __restrict__ work, int C,
         int L, const uint64_t* __restrict__ pk_ntt, uint64_t* __restrict__ ct, PrimeSet ps,
         TwSet tws) {
  extern __shared__ uint64_t lds[];
  constexpr int N = NttShape<LOGN>::N, T = NttShape<LOGN>::T;
  const int tid = threadIdx.x, l = blockIdx.x % L, m = blockIdx.x / L;
  int qi, k;
  work_pair(work, m, C, qi, k);
  const uint64_t id = qids[qi];
  int8_t* ub = reinterpret_cast<int8_t*>(lds);
  for (int b = tid; b < N / 8; b += T) {
    uint32_t o[16];
    chacha_block(K, kCpStreamU + (uint32_t)b, (uint32_t)id, (uint32_t)(id >> 32), (uint32_t)k, o);
#pragma unroll
    for (int n = 0; n < 8; ++n) ub[8 * b + n] = (int8_t)((int)(word64_of(o, n) % 3u) - 1);
  }
  __syncthreads();
  const Prime& P = ps.p[l];
  uint64_t v[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) v[a] = lift_small(ub[coef_index<LOGN>(tid, a)], P.q);
  __syncthreads();  // the transform reuses the LDS
  ntt_fwd<LOGN>(v, lds, tid, tws.tw[l], P);
  const uint64_t* pk0 = pk_ntt + ((size_t)(2 * qi) * L + l) * N;
  const uint64_t* pk1 = pk_ntt + ((size_t)(2 * qi + 1) * L + l) * N;
  uint64_t* c0 = ct + ((size_t)(2 * m) * L + l) * N;
  uint64_t* c1 = ct + ((size_t)(2 * m + 1) * L + l) * N;
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int w = ntt_slot<LOGN>(tid, a);
    c0[w] = addmod(c0[w], mulmod(v[a], pk0[w], P), P.q);
    c1[w] = addmod(c1[w], mulmod(v[a], pk1[w], P), P.q);
  }
}

// Thread per (output m, block b): the flood of coefficients 2b and 2b + 1
// (one ChaCha20 block) reduced for every limb, flood[m][l][j]; threads with
// b < N/8 also draw e1 and e2 of coefficients 8b .. 8b + 7, errs[m][c][j].
// Generated once here instead of once per limb inside the inverse transform.
__global__ void __launch_bounds__(256)
k_cp_noise(MaskKey K, const uint64_t* __restrict__ qids, const uint32_t* __restrict__ work,
           int C, long M, int N, int L, CpConst cp, DigitSet ds, PrimeSet ps,
           uint64_t* __restrict__ flood, int8_t* __restrict__ errs) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = N / 2;
  if (g >= M * nb) return;
  const int m = (int)(g / nb), b = (int)(g % nb);
  int qi, k;
  work_pair(work, m, C, qi, k);
  const uint64_t id = qids[qi];
  const uint32_t n0 = (uint32_t)id, n1 = (uint32_t)(id >> 32), n2 = (uint32_t)k;
  uint32_t o[16];
  chacha_block(K, kCpStreamFlood + (uint32_t)b, n0, n1, n2, o);
  for (int l = 0; l < L; ++l) {
    const uint64_t q = ps.p[l].q;
    ulonglong2 v;
    v.x = flood_residue(o, cp.b, cp.twob[l], ds.c[l], q);
    v.y = flood_residue(o + 8, cp.b, cp.twob[l], ds.c[l], q);
    reinterpret_cast<ulonglong2*>(flood + ((size_t)m * L + l) * N)[b] = v;
  }
  if (b < N / 8) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      chacha_block(K, (c == 0 ? kCpStreamE1 : kCpStreamE2) + (uint32_t)b, n0, n1, n2, o);
      uint32_t w0 = 0, w1 = 0;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        w0 |= (uint32_t)(uint8_t)(int8_t)cbd21(word64_of(o, n)) << (8 * n);
        w1 |= (uint32_t)(uint8_t)(int8_t)cbd21(word64_of(o, n + 4)) << (8 * n);
      }
      reinterpret_cast<uint2*>(errs + ((size_t)m * 2 + c) * N)[b] = make_uint2(w0, w1);
    }
  }
}

// k_intt_mask with the re-randomisation's coefficient-form terms (drawn by
// k_cp_noise): e1, the flood and Delta [norm - r]_t on c0, e2 on c1.
template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T, intt_mask_waves(LOGN))
k_intt_mask_cp(uint64_t* __restrict__ ct, const uint32_t* __restrict__ share,
               const uint32_t* __restrict__ norms, const uint32_t* __restrict__ work, int C,
               int L, uint32_t t, const uint64_t* __restrict__ flood,
               const int8_t* __restrict__ errs, PrimeSet ps, TwSet tws, int n, int Qa) {
  extern __shared__ uint64_t lds[];
  constexpr int N = NttShape<LOGN>::N;
  const int tid = threadIdx.x, p = intt_poly_of_block(blockIdx.x, n, Qa, C, L);
  if (p < 0) return;
  const int l = p % L, c = (p / L) & 1, m = p / (2 * L);
  const Prime& P = ps.p[l];
  uint64_t* buf = ct + (size_t)p * N;
  uint64_t v[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) v[a] = buf[ntt_slot<LOGN>(tid, a)];
  ntt_inv<LOGN>(v, lds, tid, tws.tw[l] + N, P);
  const int8_t* e = errs + ((size_t)m * 2 + c) * N;
#pragma unroll
  for (int a = 0; a < 16; ++a) v[a] = addmod(v[a], lift_small(e[coef_index<LOGN>(tid, a)], P.q), P.q);
  if (c == 0) {
    int qi, k;
    work_pair(work, m, C, qi, k);
    const uint32_t* nrm = norms + (size_t)k * N;
    const uint32_t* r = share + (size_t)m * N;
    const uint64_t* fl = flood + ((size_t)m * L + l) * N;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int j = coef_index<LOGN>(tid, a);
      const uint32_t pn = nrm[j], rj = r[j];
      const uint64_t mv = pn >= rj ? pn - rj : pn + t - rj;
      v[a] = addmod(addmod(v[a], shoup(mv, P.delta, P.deltap, P.q), P.q), fl[j], P.q);
    }
  }
  __syncthreads();  // every thread has read its inputs before any overwrite
#pragma unroll
  for (int a = 0; a < 16; ++a) buf[coef_index<LOGN>(tid, a)] = v[a];
}

// --------------------------------------------------------------------------
// fused multiply-accumulate over the resident database
// --------------------------------------------------------------------------

// Thread = one slot of one limb; it accumulates the QT x CT (query, chunk)
// pairs of its tile for both ciphertext components over all d coordinates.
// Without a tile table the schedule is every query against every chunk:
// tile y covers queries (y / ceil(C/CT)) QT .. and chunks (y mod ceil(C/CT)) CT ..,
// clamped to the last query / chunk with the clamped pairs not written.
template <int QT, int CT>
__device__ __forceinline__ MacTile<QT, CT> regular_tile(int y, int Q, int C) {
  MacTile<QT, CT> T;
  const int ncg = (C + CT - 1) / CT;
  const int q0 = (y / ncg) * QT, k0 = (y % ncg) * CT;
#pragma unroll
  for (int a = 0; a < QT; ++a) T.q[a] = q0 + a < Q ? q0 + a : Q - 1;
#pragma unroll
  for (int b = 0; b < CT; ++b) T.k[b] = k0 + b < C ? k0 + b : C - 1;
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b)
      T.out[a][b] = (q0 + a < Q && k0 + b < C) ? (q0 + a) * C + k0 + b : -1;
  return T;
}

// WIDE = false: d <= 255, a single accumulation without folded partials.
// NT: the database is streamed with nontemporal loads (read once per launch).
template <int QT, int CT, bool WIDE = true, bool NT = false>
__device__ __forceinline__ void mac_reg_slot(const MacTile<QT, CT>& T, int s, int l,
                                             const uint2* __restrict__ qntt,
                                             const uint2* __restrict__ db, int d, int L, int N,
                                             int C, const PrimeSet& ps,
                                             uint64_t* __restrict__ out) {
  const Prime& P = ps.p[l];
  const size_t qstride_i = (size_t)2 * L * N;                 // next coordinate
  const size_t dbstride_i = (size_t)N;
  const uint2* qb[QT];
  const uint2* dbb[CT];
#pragma unroll
  for (int a = 0; a < QT; ++a) qb[a] = qntt + ((size_t)T.q[a] * d * 2 * L + l) * N + s;
#pragma unroll
  for (int b = 0; b < CT; ++b) dbb[b] = db + (((size_t)l * C + T.k[b]) * d) * N + s;

  uint64_t res[QT][2][CT];
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < CT; ++b) res[a][c][b] = 0;

  // WIDE: folds of 255 coordinates added into res; otherwise one pass.
  const int step = WIDE ? 255 : d;
  for (int i0 = 0; i0 < d; i0 += step) {
    const int i1 = d - i0 < step ? d : i0 + step;
    Acc3 acc[QT][2][CT];
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < CT; ++b) acc3_zero(acc[a][c][b]);
    // Operands of coordinate i + 1 are loaded while coordinate i is
    // multiplied; the scheduling barriers keep the compiler from pulling the
    // split of the new operands (which waits for the loads) above the
    // multiplies.
    uint32_t x0[QT][2], x1[QT][2], x01[QT][2];
    uint2 yv[CT];
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const uint2 v = qb[a][i0 * qstride_i + (size_t)c * L * N];
        x0[a][c] = v.x;
        x1[a][c] = v.y;
        x01[a][c] = v.x + v.y;
      }
    auto db_load = [&](const uint2* ptr) -> uint2 {
      if constexpr (NT) {
        const uint64_t v =
            __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(ptr));
        return make_uint2(lo32(v), hi32(v));
      } else {
        return *ptr;
      }
    };
#pragma unroll
    for (int b = 0; b < CT; ++b) yv[b] = db_load(dbb[b] + i0 * dbstride_i);
    for (int i = i0; i < i1; ++i) {
      const int inext = i + 1 < i1 ? i + 1 : i;
      uint2 xn[QT][2];
      uint2 yn[CT];
#pragma unroll
      for (int a = 0; a < QT; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) xn[a][c] = qb[a][inext * qstride_i + (size_t)c * L * N];
#pragma unroll
      for (int b = 0; b < CT; ++b) yn[b] = db_load(dbb[b] + inext * dbstride_i);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        const uint2 y = yv[b];
        const uint32_t y01 = y.x + y.y;
#pragma unroll
        for (int a = 0; a < QT; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            acc[a][c][b].lo += mul32x32(x0[a][c], y.x);
            acc[a][c][b].hi += mul32x32(x1[a][c], y.y);
            acc[a][c][b].mid += mul32x32(x01[a][c], y01);
          }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int a = 0; a < QT; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          x0[a][c] = xn[a][c].x;
          x1[a][c] = xn[a][c].y;
          x01[a][c] = x0[a][c] + x1[a][c];
        }
#pragma unroll
      for (int b = 0; b < CT; ++b) yv[b] = yn[b];
    }
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < CT; ++b)
          res[a][c][b] = WIDE ? addmod(res[a][c][b], acc3_reduce(acc[a][c][b], P), P.q)
                              : acc3_reduce(acc[a][c][b], P);
    if (!WIDE) break;
  }
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int o = T.out[a][b];
      if (o < 0) continue;
#pragma unroll
      for (int c = 0; c < 2; ++c) out[(((size_t)o * 2 + c) * L + l) * N + s] = res[a][c][b];
    }
}

// Flat grid of (tile, slot range, limb) blocks.  With a tile table (work
// lists) the tile index runs fastest and the blocks are dealt to the XCDs in
// contiguous ranges (blocks are dispatched to XCDs round-robin): the
// consecutive tiles of one query group then run on one XCD at the same slot
// range and reuse that group's query operands from its L2.  The all-pairs
// schedule keeps the slot range fastest, which streams each database row
// contiguously (measured faster for a single query).
// NT (the all-pairs schedule, no tile table): each database residue is read
// once per launch, so it is streamed with nontemporal loads.
template <int QT, int CT, bool NT>
__global__ void __launch_bounds__(256)
k_mac(const uint2* __restrict__ qntt, const uint2* __restrict__ db,
      const MacTile<QT, CT>* __restrict__ tiles, int n_tiles, int Q, int d, int L, int logN,
      int C, int n_blocks, PrimeSet ps, uint64_t* __restrict__ out) {
  const int nsr = (1 << logN) / blockDim.x;
  int y, sr, l;
  if (tiles) {
    const int per_xcd = (n_blocks + 7) >> 3;
    const int lin = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (lin >= n_blocks) return;
    y = lin % n_tiles;
    sr = (lin / n_tiles) % nsr;
    l = lin / n_tiles / nsr;
  } else {
    const int lin = blockIdx.x;
    if (lin >= n_blocks) return;
    sr = lin % nsr;
    y = (lin / nsr) % n_tiles;
    l = lin / nsr / n_tiles;
  }
  const MacTile<QT, CT> T = tiles ? tiles[y] : regular_tile<QT, CT>(y, Q, C);
  mac_reg_slot<QT, CT, true, NT>(T, sr * blockDim.x + threadIdx.x, l, qntt, db, d, L, 1 << logN,
                                 C, ps, out);
}

// LDS-staged multiply-accumulate for the every-query-against-every-chunk
// schedule of a batch.  A block owns S slots of one limb, a tile of QB = QG QT
// queries and CB = CG CT chunks; per step of DI coordinates it stages the
// tile's query residues (split into 27-bit halves) and database residues in
// LDS, and each thread accumulates its QT x CT register tile for one slot.
// Blocks are numbered so that every XCD (blocks b with equal b mod 8) walks
// its own range of (slot tile, limb) pairs, all query/chunk tiles of a pair
// running back to back, which keeps the pair's operands in that XCD's L2.
// Fold of the accumulators into residues and the write of the block's
// outputs (pairs whose query or chunk index falls outside the batch are
// padding and are not written).
template <int QT, int CT>
__device__ __forceinline__ void mac_store(const Acc3 (&acc)[QT][2][CT],
                                          const uint64_t (&res)[QT][2][CT], bool have_res,
                                          const Prime& P, int q0, int k0,
                                          int gq, int gc, int Q, int C, int L, int l, int N,
                                          int slot, uint64_t* __restrict__ out) {
#pragma unroll
  for (int a = 0; a < QT; ++a) {
    const int q = q0 + gq * QT + a;
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int k = k0 + gc * CT + b;
      if (q >= Q || k >= C) continue;
      const size_t o = (size_t)q * C + k;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint64_t v = acc3_reduce(acc[a][c][b], P);
        if (have_res) v = addmod(v, res[a][c][b], P.q);
        out[((o * 2 + c) * L + l) * N + slot] = v;
      }
    }
  }
}

// WIDE: d > FOLD, partial residues of earlier folds are kept in registers.
template <int QT, int CT, int QG, int CG, int S, int DI, int UNR, bool WIDE>
__global__ void __launch_bounds__(S * QG * CG)
k_mac_lds(const uint2* __restrict__ qntt, const uint2* __restrict__ db, int Q, int d, int L,
          int logN, int C, int n_blocks, PrimeSet ps, uint64_t* __restrict__ out) {
  constexpr int QB = QT * QG, CB = CT * CG, NT = S * QG * CG;
  constexpr int FOLD = (255 / DI) * DI;  // coordinates per 64-bit accumulation
  constexpr int QE = QB * 2 * DI * S, DE = CB * DI * S;  // staged words per step
  constexpr int NQE = (QE + NT - 1) / NT, NDE = (DE + NT - 1) / NT;
  __shared__ uint2 sq[2][QE];
  __shared__ uint2 sd[2][DE];
  const int N = 1 << logN;
  const int nqt = (Q + QB - 1) / QB, nct = (C + CB - 1) / CB;
  // XCD-aware decode of the flat block index
  const int per_xcd = (n_blocks + 7) >> 3;
  const int lin = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lin >= n_blocks) return;
  const int y = lin % (nqt * nct);
  const int sl = lin / (nqt * nct);
  const int l = sl % L, st = sl / L;
  const int q0 = (y % nqt) * QB, k0 = (y / nqt) * CB;
  const int s0 = st * S;
  const Prime& P = ps.p[l];
  const int tid = threadIdx.x;
  const int s = tid % S, g = tid / S, gq = g % QG, gc = g / QG;

  // Staging: thread tid moves words e = tid + u NT of every step.  Their
  // source addresses for coordinate 0 are computed once; a step at
  // coordinate i0 adds i0 times the per-coordinate stride.
  const uint2* qsrc[NQE];
  int qdi[NQE];
  const uint2* dsrc[NDE];
  int ddi[NDE];
#pragma unroll
  for (int u = 0; u < NQE; ++u) {
    const int e = tid + u * NT < QE ? tid + u * NT : QE - 1;
    const int ss = e % S, r = e / S;
    const int di = r % DI, qc = r / DI;
    const int c = qc & 1, qq = qc >> 1;
    const int q = q0 + qq < Q ? q0 + qq : Q - 1;
    qdi[u] = tid + u * NT < QE ? di : 1 << 30;
    qsrc[u] = qntt + ((((size_t)q * d + di) * 2 + c) * L + l) * N + s0 + ss;
  }
#pragma unroll
  for (int u = 0; u < NDE; ++u) {
    const int e = tid + u * NT < DE ? tid + u * NT : DE - 1;
    const int ss = e % S, r = e / S;
    const int di = r % DI, cc = r / DI;
    const int k = k0 + cc < C ? k0 + cc : C - 1;
    ddi[u] = tid + u * NT < DE ? di : 1 << 30;
    dsrc[u] = db + (((size_t)l * C + k) * d + di) * N + s0 + ss;
  }
  const size_t qstep = (size_t)2 * L * N, dstep = (size_t)N;

  // Two register sets ring the staged words: while LDS buffer `cur` is
  // multiplied, the words of the next step are on their way into LDS buffer
  // cur ^ 1 and those of the step after next are already being loaded.
  uint2 rqA[NQE], rqB[NQE];
  uint2 rdA[NDE], rdB[NDE];
  auto fetch = [&](int i0, uint2 (&rq)[NQE], uint2 (&rd)[NDE]) {
#pragma unroll
    for (int u = 0; u < NQE; ++u)
      rq[u] = i0 + qdi[u] < d ? qsrc[u][(size_t)i0 * qstep] : make_uint2(0u, 0u);
#pragma unroll
    for (int u = 0; u < NDE; ++u)
      rd[u] = i0 + ddi[u] < d ? dsrc[u][(size_t)i0 * dstep] : make_uint2(0u, 0u);
  };
  auto stash = [&](int buf, const uint2 (&rq)[NQE], const uint2 (&rd)[NDE]) {
#pragma unroll
    for (int u = 0; u < NQE; ++u) {
      const int e = tid + u * NT;
      if (e < QE) sq[buf][e] = rq[u];
    }
#pragma unroll
    for (int u = 0; u < NDE; ++u) {
      const int e = tid + u * NT;
      if (e < DE) sd[buf][e] = rd[u];
    }
  };

  Acc3 acc[QT][2][CT];
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < CT; ++b) acc3_zero(acc[a][c][b]);
  uint64_t res[QT][2][CT];
  if (WIDE) {
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < CT; ++b) res[a][c][b] = 0;
  }

  auto compute = [&](int cur) {
#pragma unroll UNR
    for (int di = 0; di < DI; ++di) {
      uint32_t x0[QT][2], x1[QT][2], x01[QT][2];
#pragma unroll
      for (int a = 0; a < QT; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const uint2 v = sq[cur][(((gq * QT + a) * 2 + c) * DI + di) * S + s];
          x0[a][c] = v.x;
          x1[a][c] = v.y;
          x01[a][c] = v.x + v.y;
        }
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        const uint2 yv = sd[cur][((gc * CT + b) * DI + di) * S + s];
        const uint32_t y01 = yv.x + yv.y;
#pragma unroll
        for (int a = 0; a < QT; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            acc[a][c][b].lo += mul32x32(x0[a][c], yv.x);
            acc[a][c][b].hi += mul32x32(x1[a][c], yv.y);
            acc[a][c][b].mid += mul32x32(x01[a][c], y01);
          }
      }
    }
  };
  auto fold = [&](int i0) {
    if (WIDE && i0 + DI < d && (i0 + DI) % FOLD == 0) {
#pragma unroll
      for (int a = 0; a < QT; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int b = 0; b < CT; ++b) {
            res[a][c][b] = addmod(res[a][c][b], acc3_reduce(acc[a][c][b], P), P.q);
            acc3_zero(acc[a][c][b]);
          }
    }
  };

  fetch(0, rqA, rdA);
  if (DI < d) fetch(DI, rqB, rdB);
  stash(0, rqA, rdA);
  __syncthreads();
  int cur = 0;
  for (int i0 = 0; i0 < d; i0 += 2 * DI) {
    // step at i0: LDS[cur] holds it, set B holds i0 + DI
    if (i0 + 2 * DI < d) fetch(i0 + 2 * DI, rqA, rdA);
    __builtin_amdgcn_sched_barrier(0);
    compute(cur);
    __builtin_amdgcn_sched_barrier(0);
    fold(i0);
    if (i0 + DI >= d) break;
    stash(cur ^ 1, rqB, rdB);
    __syncthreads();
    cur ^= 1;
    // step at i0 + DI: LDS[cur] holds it, set A holds i0 + 2 DI
    if (i0 + 3 * DI < d) fetch(i0 + 3 * DI, rqB, rdB);
    __builtin_amdgcn_sched_barrier(0);
    compute(cur);
    __builtin_amdgcn_sched_barrier(0);
    fold(i0 + DI);
    if (i0 + 2 * DI >= d) break;
    stash(cur ^ 1, rqA, rdA);
    __syncthreads();
    cur ^= 1;
  }
  mac_store<QT, CT>(acc, res, WIDE, P, q0, k0, gq, gc, Q, C, L, l, N, s0 + s, out);
}

// Direct-to-LDS variant of k_mac_lds: the staged words go from global
// memory straight into LDS (global_load_lds, 16 bytes per lane), so no
// registers are spent on staging and the query words arrive already split.
// LDS buffer B0/B1 alternate: the next step is loaded into one while the
// other is multiplied.
// LDS footprint of one direct-to-LDS tile: two query and two database buffers.
template <int QT, int CT, int QG, int CG, int S, int DI>
struct MacDlShape {
  static constexpr int QU = QT * QG * 2 * DI * (S / 2), DU = CT * CG * DI * (S / 2);
  static constexpr size_t lds_bytes = (size_t)2 * (QU + DU) * sizeof(uint4);
};

// Tile lin of the all-pairs schedule (query tile fastest, then chunk tile,
// then limb, then slot range), computed by the NT = S QG CG threads of a
// workgroup with the given LDS buffers.
template <int QT, int CT, int QG, int CG, int S, int DI, int UNR, bool WIDE>
__device__ __forceinline__ void mac_dl_tile(int lin, int tid, uint4* sq0, uint4* sq1, uint4* sd0,
                                            uint4* sd1, const uint2* __restrict__ qntt,
                                            const uint2* __restrict__ db, int Q, int d, int L,
                                            int logN, int C, const PrimeSet& ps,
                                            uint64_t* __restrict__ out) {
  constexpr int QB = QT * QG, CB = CT * CG, NT = S * QG * CG;
  constexpr int FOLD = (255 / DI) * DI;
  constexpr int H = S / 2;                            // 16-byte units per row of S slots
  constexpr int QU = QB * 2 * DI * H, DU = CB * DI * H;  // 16-byte units per step
  constexpr int NQU = (QU + NT - 1) / NT, NDU = (DU + NT - 1) / NT;
  const int N = 1 << logN;
  const int nqt = (Q + QB - 1) / QB, nct = (C + CB - 1) / CB;
  const int y = lin % (nqt * nct);
  const int sl = lin / (nqt * nct);
  const int l = sl % L, st = sl / L;
  const int q0 = (y % nqt) * QB, k0 = (y / nqt) * CB;
  const int s0 = st * S;
  const Prime& P = ps.p[l];
  const int s = tid % S, g = tid / S, gq = g % QG, gc = g / QG;
  const int wbase = __builtin_amdgcn_readfirstlane(tid) & ~63;

  const uint2* qsrc[NQU];
  int qdi[NQU];
  const uint2* dsrc[NDU];
  int ddi[NDU];
#pragma unroll
  for (int u = 0; u < NQU; ++u) {
    const int e = tid + u * NT;
    const int ee = e < QU ? e : 0;
    const int pr = ee % H, r = ee / H;
    const int di = r % DI, qc = r / DI;
    const int c = qc & 1, qq = qc >> 1;
    const int q = q0 + qq < Q ? q0 + qq : Q - 1;
    qdi[u] = e < QU ? di : 1 << 30;
    qsrc[u] = qntt + ((((size_t)q * d + di) * 2 + c) * L + l) * N + s0 + 2 * pr;
  }
#pragma unroll
  for (int u = 0; u < NDU; ++u) {
    const int e = tid + u * NT;
    const int ee = e < DU ? e : 0;
    const int pr = ee % H, r = ee / H;
    const int di = r % DI, cc = r / DI;
    const int k = k0 + cc < C ? k0 + cc : C - 1;
    ddi[u] = e < DU ? di : 1 << 30;
    dsrc[u] = db + (((size_t)l * C + k) * d + di) * N + s0 + 2 * pr;
  }
  const size_t qstep = (size_t)2 * L * N, dstep = (size_t)N;
  auto issue = [&](int i0, uint4* bq, uint4* bd) {
#pragma unroll
    for (int u = 0; u < NQU; ++u)
      if (i0 + qdi[u] < d)
        __builtin_amdgcn_global_load_lds(
            (const void*)(qsrc[u] + (size_t)i0 * qstep),
            (__attribute__((address_space(3))) void*)(bq + wbase + u * NT), 16, 0, 0);
#pragma unroll
    for (int u = 0; u < NDU; ++u)
      if (i0 + ddi[u] < d)
        __builtin_amdgcn_global_load_lds(
            (const void*)(dsrc[u] + (size_t)i0 * dstep),
            (__attribute__((address_space(3))) void*)(bd + wbase + u * NT), 16, 0, 0);
  };

  Acc3 acc[QT][2][CT];
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < CT; ++b) acc3_zero(acc[a][c][b]);
  uint64_t res[QT][2][CT];
  if (WIDE) {
#pragma unroll
    for (int a = 0; a < QT; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < CT; ++b) res[a][c][b] = 0;
  }
  // Threads whose whole chunk group lies past the last chunk (the padding of
  // a ragged final chunk tile) still stage loads and meet the barriers but
  // skip the multiply-adds; the group is uniform over a wavefront when
  // S QG is a multiple of 64, so those waves free their ALU slots.
  const bool idle = k0 + gc * CT >= C;
  auto compute = [&](const uint4* bq4, const uint4* bd4, int ndi) {
    if (idle) return;
    const uint2* bq = reinterpret_cast<const uint2*>(bq4);
    const uint2* bd = reinterpret_cast<const uint2*>(bd4);
#pragma unroll UNR
    for (int di = 0; di < ndi; ++di) {
      uint32_t x0[QT][2], x1[QT][2], x01[QT][2];
#pragma unroll
      for (int a = 0; a < QT; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const uint2 v = bq[(((gq * QT + a) * 2 + c) * DI + di) * S + s];
          x0[a][c] = v.x;
          x1[a][c] = v.y;
          x01[a][c] = v.x + v.y;
        }
#pragma unroll
      for (int b = 0; b < CT; ++b) {
        const uint2 yv = bd[((gc * CT + b) * DI + di) * S + s];
        const uint32_t y01 = yv.x + yv.y;
#pragma unroll
        for (int a = 0; a < QT; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            acc[a][c][b].lo += mul32x32(x0[a][c], yv.x);
            acc[a][c][b].hi += mul32x32(x1[a][c], yv.y);
            acc[a][c][b].mid += mul32x32(x01[a][c], y01);
          }
      }
    }
  };
  auto fold = [&](int i0) {
    if (WIDE && i0 + DI < d && (i0 + DI) % FOLD == 0) {
#pragma unroll
      for (int a = 0; a < QT; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int b = 0; b < CT; ++b) {
            res[a][c][b] = addmod(res[a][c][b], acc3_reduce(acc[a][c][b], P), P.q);
            acc3_zero(acc[a][c][b]);
          }
    }
  };

  issue(0, sq0, sd0);
  __builtin_amdgcn_s_waitcnt(0);  // all counters: the first step has landed
  __syncthreads();
  for (int i0 = 0; i0 < d; i0 += 2 * DI) {
    if (i0 + DI < d) issue(i0 + DI, sq1, sd1);
    compute(sq0, sd0, d - i0 < DI ? d - i0 : DI);
    fold(i0);
    if (i0 + DI >= d) break;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (i0 + 2 * DI < d) issue(i0 + 2 * DI, sq0, sd0);
    compute(sq1, sd1, d - i0 - DI < DI ? d - i0 - DI : DI);
    fold(i0 + DI);
    if (i0 + 2 * DI >= d) break;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  mac_store<QT, CT>(acc, res, WIDE, P, q0, k0, gq, gc, Q, C, L, l, N, s0 + s, out);
}

template <int QT, int CT, int QG, int CG, int S, int DI, int UNR, bool WIDE>
__global__ void __launch_bounds__(S * QG * CG)
k_mac_dl(const uint2* __restrict__ qntt, const uint2* __restrict__ db, int Q, int d, int L,
         int logN, int C, int n_blocks, PrimeSet ps, uint64_t* __restrict__ out) {
  using SH = MacDlShape<QT, CT, QG, CG, S, DI>;
  __shared__ uint4 sq0[SH::QU], sq1[SH::QU];
  __shared__ uint4 sd0[SH::DU], sd1[SH::DU];
  const int per_xcd = (n_blocks + 7) >> 3;
  const int lin = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lin >= n_blocks) return;
  mac_dl_tile<QT, CT, QG, CG, S, DI, UNR, WIDE>(lin, threadIdx.x, sq0, sq1, sd0, sd1, qntt, db,
                                                Q, d, L, logN, C, ps, out);
}

// --------------------------------------------------------------------------
// the whole batch as one persistent launch
// --------------------------------------------------------------------------

// Control words of the persistent schedule (zeroed before each launch).
enum : int {
  kTicket1 = 0,   // query NTT and mask-row items
  kTicketMac = 1, // eight multiply-accumulate queues, one per XCD
  kTicket3 = 9,   // INTT + mask items
  kDoneNtt = 10,
  kDoneMasks = 11,
  kDoneMac = 12,
  kAbort = 13,
  kCtrlWords = kPersistCtrlWords
};
constexpr uint32_t kSpinLimit = 1u << 25;  // about 7 s of 200 ns sleeps

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}


// Physical XCD of the calling wave (hardware register XCC_ID, bits 0..3).
__device__ __forceinline__ int xcd_id() {
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u);
}

// Thread 0 waits until ctrl[idx] >= target (acquire); false on abort or
// time-out, which also raises the abort word so that every waiter leaves.
__device__ bool wait_at_least(uint32_t* ctrl, int idx, uint32_t target, uint32_t* err) {
  for (uint32_t spins = 0;; ++spins) {
    if (__hip_atomic_load(ctrl + idx, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target)
      return true;
    if (__hip_atomic_load(ctrl + kAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (spins >= kSpinLimit) {
      atomicOr(err, 4u);
      __hip_atomic_store(ctrl + kAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(8);
  }
}

// Needs d <= (255 / DI) DI (one accumulation pass per tile).
// Work items, in ticket order (an item only depends on items of earlier
// phases, so the schedule needs no co-residency and cannot deadlock):
//   phase 1: forward NTT of each query polynomial, then each output row's
//            masks (no dependencies);
//   phase 2: multiply-accumulate tiles, split into eight contiguous ranges
//            served first to the blocks of the matching XCD (so that the
//            query tiles sharing a database tile share that XCD's L2), then
//            stolen by any block;
//   phase 3: INTT + mask of each output polynomial.
// A block publishes how many items of a phase it finished (one device-wide
// release) when it leaves the phase, and waits (one acquire) for the counts
// a phase depends on when it enters it.
template <int LOGN, int QT, int CT, int QG, int CG, int DI, int TQT, int TCT>
__global__ void __launch_bounds__(NttShape<LOGN>::T, 4)
k_persistent(PersistArgs A, PrimeSet ps, TwSet tws) {
  constexpr int T = NttShape<LOGN>::T, N = NttShape<LOGN>::N;
  constexpr int S = T / (QG * CG);
  using SH = MacDlShape<QT, CT, QG, CG, S, DI>;
  static_assert(S * QG * CG == T && S >= 2, "tile does not match the workgroup");
  extern __shared__ uint64_t lds[];
  __shared__ int s_ticket, s_ok;
  const int tid = threadIdx.x;
  uint32_t* ctrl = A.ctrl;
  const int L = A.L;
  const int n_ntt = A.Q * A.d * 2 * L;
  const int n1 = n_ntt + A.M;

  // ---- phase 1
  uint32_t done_ntt = 0, done_masks = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_ticket = (int)atomicAdd(ctrl + kTicket1, 1u);
    __syncthreads();
    const int tk = s_ticket;
    if (tk >= n1) break;
    if (tk < n_ntt) {
      ntt_fwd_poly<LOGN, 1>(tk, tid, lds, A.ct_in, A.qntt, L, ps, tws, A.err);
      ++done_ntt;
    } else {
      const int m = tk - n_ntt;
      int qi, k;
      work_pair(A.work, m, A.C, qi, k);
      const uint64_t id = A.qids[qi];
      for (int b = tid; b < (N >> 2); b += T)
        mask_block(A.K, id, k, b, A.t, A.tone, A.share + (size_t)m * N);
      ++done_masks;
    }
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    if (done_ntt) atomicAdd(ctrl + kDoneNtt, done_ntt);
    if (done_masks) atomicAdd(ctrl + kDoneMasks, done_masks);
    s_ok = wait_at_least(ctrl, kDoneNtt, (uint32_t)n_ntt, A.err);
  }
  __syncthreads();
  if (!s_ok) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

  // ---- phase 2
  const uint2* qn = reinterpret_cast<const uint2*>(A.qntt);
  uint4* sq0 = reinterpret_cast<uint4*>(lds);
  uint4* sq1 = sq0 + SH::QU;
  uint4* sd0 = sq1 + SH::QU;
  uint4* sd1 = sd0 + SH::DU;
  int n_mac;
  if (A.work) {
    n_mac = A.n_tiles * (N / T) * L;
  } else {
    const int nqt = (A.Q + QT * QG - 1) / (QT * QG), nct = (A.C + CT * CG - 1) / (CT * CG);
    n_mac = nqt * nct * L * (N / S);
  }
  const int per_q = (n_mac + 7) >> 3;
  const int home = xcd_id();
  uint32_t done_mac = 0;
  for (int j = 0; j < 8; ++j) {
    const int x = (home + j) & 7;
    const int lo = x * per_q, hi = min(n_mac, lo + per_q);
    for (;;) {
      __syncthreads();
      if (tid == 0) s_ticket = lo + (int)atomicAdd(ctrl + kTicketMac + x, 1u);
      __syncthreads();
      const int lin = s_ticket;
      if (lin >= hi) break;
      if (A.work) {
        // (tile, slot range, limb), slot range fastest
        const int r = lin % (N / T), jl = lin / (N / T);
        const int tile = jl % A.n_tiles, l = jl / A.n_tiles;
        const MacTile<TQT, TCT> Tl =
            reinterpret_cast<const MacTile<TQT, TCT>*>(A.tiles)[tile];
        mac_reg_slot<TQT, TCT, false>(Tl, r * T + tid, l, qn, A.db, A.d, L, N, A.C, ps,
                                      A.ct_out);
      } else {
        mac_dl_tile<QT, CT, QG, CG, S, DI, 1, false>(lin, tid, sq0, sq1, sd0, sd1, qn, A.db,
                                                     A.Q, A.d, L, LOGN, A.C, ps, A.ct_out);
      }
      ++done_mac;
    }
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    if (done_mac) atomicAdd(ctrl + kDoneMac, done_mac);
    s_ok = wait_at_least(ctrl, kDoneMac, (uint32_t)n_mac, A.err) &&
           wait_at_least(ctrl, kDoneMasks, (uint32_t)A.M, A.err);
  }
  __syncthreads();
  if (!s_ok) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

  // ---- phase 3
  const int n3 = A.M * 2 * L;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_ticket = (int)atomicAdd(ctrl + kTicket3, 1u);
    __syncthreads();
    const int tk = s_ticket;
    if (tk >= n3) break;
    intt_mask_poly<LOGN>(tk, tid, lds, A.ct_out, A.share, A.norms, A.work, A.C, L, A.t, ps, tws);
  }
}

// --------------------------------------------------------------------------
// database encoding
// --------------------------------------------------------------------------

// Thread per slot: gathers the slot's point into the transposed plaintext
// buffer gt[k][i][j] = -2 p[i] (int16) and writes [||p||^2] to norms.
// Slots [base, base + total) of the database; gt is local to that range.
__global__ void __launch_bounds__(256)
k_gather(const uint8_t* __restrict__ pts, int is_signed, long n, int d,
         const int64_t* __restrict__ slot_point, long base, long total, int logN,
         int16_t* __restrict__ gt, uint32_t* __restrict__ norms, uint32_t* err) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N = 1 << logN;
  const long k = g >> logN;
  const int j = (int)(g & (N - 1));
  long pid = slot_point[base + g];
  if (pid >= n || pid < -1) {
    if (err) atomicOr(err, 2u);
    pid = -1;
  }
  int16_t* col = gt + (size_t)k * d * N + j;
  uint32_t nrm = 0;
  if (pid < 0) {
    for (int i = 0; i < d; ++i) col[(size_t)i * N] = 0;
  } else {
    const uint8_t* row = pts + (size_t)pid * d;
    for (int i = 0; i < d; ++i) {
      const int x = is_signed ? (int)(int8_t)row[i] : (int)row[i];
      col[(size_t)i * N] = (int16_t)(-2 * x);
      nrm += (uint32_t)(x * x);
    }
  }
  norms[base + g] = nrm;
}

// Gathered chunks of one call (per-query chunks of retrieved points): as
// k_gather, into 32-bit plaintext coefficients, for kind 0 / 1 (uint8 /
// int8 points: -2 p[i] and ||p||^2) or kind 2: the server's additive shares
// p_s in [0, t) of secret-shared points and of their squared norms, where the
// coefficient is the centred representative of -2 p_s mod t in
// (-t/2, t/2] and the norm plane holds the norm share.  A share >= t sets
// error bit 8 and is taken as 0.
__global__ void __launch_bounds__(256)
k_gather32(const void* __restrict__ pts, int kind, long n, int d,
           const uint32_t* __restrict__ norm_shares, uint32_t t,
           const int64_t* __restrict__ slot_point, long base, long total, int logN,
           int32_t* __restrict__ gt, uint32_t* __restrict__ norms, uint32_t* err) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N = 1 << logN;
  const long k = g >> logN;
  const int j = (int)(g & (N - 1));
  long pid = slot_point[base + g];
  if (pid >= n || pid < -1) {
    if (err) atomicOr(err, 2u);
    pid = -1;
  }
  int32_t* col = gt + (size_t)k * d * N + j;
  uint32_t nrm = 0;
  bool bad = false;
  if (pid < 0) {
    for (int i = 0; i < d; ++i) col[(size_t)i * N] = 0;
  } else if (kind == 2) {
    const uint32_t* row = reinterpret_cast<const uint32_t*>(pts) + (size_t)pid * d;
    for (int i = 0; i < d; ++i) {
      uint32_t x = row[i];
      if (x >= t) {
        bad = true;
        x = 0;
      }
      const uint64_t two = (2ull * x) % t;
      int64_t v = two ? (int64_t)t - (int64_t)two : 0;  // -2 x mod t in [0, t)
      if (v > (int64_t)(t / 2)) v -= t;
      col[(size_t)i * N] = (int32_t)v;
    }
    nrm = norm_shares[pid];
    if (nrm >= t) {
      bad = true;
      nrm = 0;
    }
  } else {
    const uint8_t* row = reinterpret_cast<const uint8_t*>(pts) + (size_t)pid * d;
    for (int i = 0; i < d; ++i) {
      const int x = kind == 1 ? (int)(int8_t)row[i] : (int)row[i];
      col[(size_t)i * N] = -2 * x;
      nrm += (uint32_t)(x * x);
    }
  }
  if (bad && err) atomicOr(err, 8u);
  norms[base + g] = nrm;
}

// Workgroup per (l, k, i) with k in [k0, k0 + nk): lift the signed
// plaintext row mod q_l, forward NTT, store as 27-bit halves.
template <int LOGN, typename G>
__global__ void __launch_bounds__(NttShape<LOGN>::T, 4)
k_encode_ntt(const G* __restrict__ gt, uint2* __restrict__ dbres, int k0, int nk, int C,
             int d, int L, PrimeSet ps, TwSet tws) {
  extern __shared__ uint64_t lds[];
  constexpr int N = NttShape<LOGN>::N;
  const int tid = threadIdx.x;
  const long bl = blockIdx.x;  // (l nk + k - k0) d + i
  const int l = (int)(bl / ((long)nk * d));
  const long ki = bl % ((long)nk * d);
  const long b = ((long)l * C + k0) * d + ki;
  const Prime& P = ps.p[l];
  const G* src = gt + (size_t)ki * N;
  uint64_t v[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int64_t x = src[coef_index<LOGN>(tid, a)];
    v[a] = x < 0 ? P.q - (uint64_t)(-x) : (uint64_t)x;
  }
  ntt_fwd<LOGN>(v, lds, tid, tws.tw[l], P);
  uint2* dst = dbres + (size_t)b * N;
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    uint2 y;
    split27(v[a], y.x, y.y);
    dst[ntt_slot<LOGN>(tid, a)] = y;
  }
}

// --------------------------------------------------------------------------
// client helpers: secret key transform, encryption, decryption
// --------------------------------------------------------------------------

// Workgroup per limb: NTT of the ternary secret lifted mod q_l.
template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T)
k_sk_ntt(const int8_t* __restrict__ sk, uint64_t* __restrict__ out, PrimeSet ps, TwSet tws) {
  extern __shared__ uint64_t lds[];
  constexpr int N = NttShape<LOGN>::N;
  const int tid = threadIdx.x, l = blockIdx.x;
  const Prime& P = ps.p[l];
  uint64_t v[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int x = sk[coef_index<LOGN>(tid, a)];
    v[a] = x < 0 ? P.q - (uint64_t)(-x) : (uint64_t)x;
  }
  ntt_fwd<LOGN>(v, lds, tid, tws.tw[l], P);
#pragma unroll
  for (int a = 0; a < 16; ++a) out[(size_t)l * N + ntt_slot<LOGN>(tid, a)] = v[a];
}

// --------------------------------------------------------------------------
// client randomness drawn from a seed (key generation and encryption helpers):
// ChaCha20 with key (seed low word, seed high word, purpose, 0, ..., 0),
// purpose 1 secret key, 2 uniform component a, 3 error e, 4 and 5 the same for
// the public key
// --------------------------------------------------------------------------

__device__ __forceinline__ MaskKey client_key(uint64_t seed, uint32_t purpose) {
  MaskKey K;
  K.k[0] = (uint32_t)seed;
  K.k[1] = (uint32_t)(seed >> 32);
  K.k[2] = purpose;
#pragma unroll
  for (int i = 3; i < 8; ++i) K.k[i] = 0;
  return K;
}

// (w3 2^96 + w2 2^64 + w1 2^32 + w0) mod q for q < 2^54: Horner steps of one
// byte, every intermediate below 2^62.
__device__ uint64_t mod_q_128(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint64_t q) {
  const uint32_t w[4] = {w3, w2, w1, w0};
  uint64_t r = 0;
  for (int a = 0; a < 4; ++a)
    for (int sh = 24; sh >= 0; sh -= 8) r = ((r << 8) | ((w[a] >> sh) & 0xFFu)) % q;
  return r;
}

// Thread per block b (coefficients 8b .. 8b+7): s_j = (x_j mod 3) - 1 with
// x_j the 64-bit word j % 8 of block j / 8, nonce (0, 0, 0).
__global__ void __launch_bounds__(256) k_keygen(uint64_t seed, int N, int8_t* __restrict__ sk) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= N / 8) return;
  const MaskKey K = client_key(seed, 1);
  uint32_t o[16];
  chacha_block(K, (uint32_t)b, 0u, 0u, 0u, o);
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const uint64_t x = (uint64_t)o[2 * n] | (uint64_t)o[2 * n + 1] << 32;
    sk[8 * b + n] = (int8_t)((int)(x % 3u) - 1);
  }
}

// Thread per (query x coordinate qd, limb l, block b): a_j for j = 4b .. 4b+3
// is the 128-bit integer of words 4(j%4) .. 4(j%4)+3 of block b, nonce
// (query, coordinate, limb), reduced mod q_l.  a: [Qd][L][N].
__global__ void __launch_bounds__(256)
k_sample_a(uint64_t seed, uint32_t purpose, int d, int L, int N, long total, PrimeSet ps,
           uint64_t* __restrict__ a) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int nb = N / 4;
  const int b = (int)(g % nb);
  const long r = g / nb;
  const int l = (int)(r % L);
  const long qd = r / L;
  const MaskKey K = client_key(seed, purpose);
  uint32_t o[16];
  chacha_block(K, (uint32_t)b, (uint32_t)(qd / d), (uint32_t)(qd % d), (uint32_t)l, o);
  const uint64_t q = ps.p[l].q;
  uint64_t* row = a + ((size_t)qd * L + l) * N + 4 * b;
#pragma unroll
  for (int n = 0; n < 4; ++n)
    row[n] = mod_q_128(o[4 * n], o[4 * n + 1], o[4 * n + 2], o[4 * n + 3], q);
}

// Thread per (query x coordinate qd, block b): centred binomial error
// (eta = 21) e_j = popcount(bits 0..20 of x_j) - popcount(bits 21..41 of x_j),
// x_j the 64-bit word j % 8 of block j / 8, nonce (query, coordinate, 0).
__global__ void __launch_bounds__(256)
k_sample_e(uint64_t seed, uint32_t purpose, int d, int N, long total, int16_t* __restrict__ e) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int nb = N / 8;
  const int b = (int)(g % nb);
  const long qd = g / nb;
  const MaskKey K = client_key(seed, purpose);
  uint32_t o[16];
  chacha_block(K, (uint32_t)b, (uint32_t)(qd / d), (uint32_t)(qd % d), 0u, o);
  int16_t* row = e + (size_t)qd * N + 8 * b;
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const uint64_t x = (uint64_t)o[2 * n] | (uint64_t)o[2 * n + 1] << 32;
    row[n] = (int16_t)(__popcll(x & 0x1FFFFFull) - __popcll((x >> 21) & 0x1FFFFFull));
  }
}

// Workgroup per (query, coordinate, limb): c1 = a, c0 = -a s + e + Delta m.
template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T)
k_encrypt(const uint64_t* __restrict__ a_in, const int16_t* __restrict__ e_in,
          const int32_t* __restrict__ msgs, const uint64_t* __restrict__ sk_ntt,
          uint64_t* __restrict__ ct, int L, uint32_t t, PrimeSet ps, TwSet tws) {
  extern __shared__ uint64_t lds[];
  constexpr int N = NttShape<LOGN>::N;
  const int tid = threadIdx.x;
  const int b = blockIdx.x;  // (qi d + i) L + l
  const int l = b % L;
  const int qd = b / L;      // qi d + i
  const Prime& P = ps.p[l];
  const uint64_t* a = a_in + (size_t)b * N;
  uint64_t v[16];
#pragma unroll
  for (int x = 0; x < 16; ++x) v[x] = a[coef_index<LOGN>(tid, x)];
  ntt_fwd<LOGN>(v, lds, tid, tws.tw[l], P);
#pragma unroll
  for (int x = 0; x < 16; ++x)
    v[x] = mulmod(v[x], sk_ntt[(size_t)l * N + ntt_slot<LOGN>(tid, x)], P);
  ntt_inv<LOGN>(v, lds, tid, tws.tw[l] + N, P);
  // message [m]_t as a constant: Delta m in coefficient 0
  const int64_t mraw = msgs[qd];
  int64_t mm = mraw % (int64_t)t;
  if (mm < 0) mm += t;
  const uint64_t dm = shoup((uint64_t)mm, P.delta, P.deltap, P.q);
  const int16_t* e = e_in + (size_t)qd * N;
  uint64_t* c0 = ct + ((size_t)qd * 2 * L + l) * N;
  uint64_t* c1 = ct + (((size_t)qd * 2 + 1) * L + l) * N;
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    const int j = coef_index<LOGN>(tid, x);
    const int ej = e[j];
    const uint64_t ev = ej < 0 ? P.q - (uint64_t)(-ej) : (uint64_t)ej;
    uint64_t r = submod(ev, v[x], P.q);
    if (j == 0) r = addmod(r, dm, P.q);
    c0[j] = r;
  }
  for (int j = tid; j < N; j += blockDim.x) c1[j] = a[j];
}

// Multi-word helpers for the exact CRT decode (little-endian 32-bit words).
__device__ __forceinline__ void mw_addmul(uint32_t (&z)[kMaxWords], const uint32_t* m,
                                          uint32_t b, int shift_words, int words) {
  uint64_t carry = 0;
  for (int w = 0; w + shift_words < kMaxWords; ++w) {
    const uint32_t mw = w < words ? m[w] : 0u;
    const uint64_t cur = (uint64_t)z[w + shift_words] + (uint64_t)mw * b + carry;
    z[w + shift_words] = (uint32_t)cur;
    carry = cur >> 32;
  }
}

// z >= y ?
__device__ __forceinline__ bool mw_geq(const uint32_t (&z)[kMaxWords],
                                       const uint32_t (&y)[kMaxWords]) {
  bool gt = false, eq = true;
  for (int w = kMaxWords - 1; w >= 0; --w) {
    if (eq) {
      if (z[w] > y[w]) { gt = true; eq = false; }
      else if (z[w] < y[w]) { eq = false; }
    }
  }
  return gt || eq;
}

__device__ __forceinline__ void mw_sub(uint32_t (&z)[kMaxWords], const uint32_t (&y)[kMaxWords]) {
  int64_t borrow = 0;
  for (int w = 0; w < kMaxWords; ++w) {
    const int64_t cur = (int64_t)z[w] - (int64_t)y[w] - borrow;
    z[w] = (uint32_t)cur;
    borrow = cur < 0 ? 1 : 0;
  }
}

// m = round(t x / q) mod t for x given by its residues xl (exact):
//   y_l = x_l (q/q_l)^-1 mod q_l,  y_l t = A_l q_l + B_l,
//   t x / q = sum_l A_l + sum_l B_l / q_l  (mod t),
//   round(sum_l B_l / q_l) = floor((2 Z + q) / 2q),  Z = sum_l B_l (q / q_l).
__device__ __forceinline__ uint32_t crt_round(const uint64_t* xl, int L, const PrimeSet& ps,
                                              const DecodeConst& D) {
  uint32_t Z[kMaxWords];
#pragma unroll
  for (int w = 0; w < kMaxWords; ++w) Z[w] = 0;
  uint64_t sumA = 0;
  for (int l = 0; l < L; ++l) {
    const Prime& P = ps.p[l];
    const uint64_t y = shoup(xl[l], D.inv[l], D.invp[l], P.q);
    uint64_t A = mulhi64(y, D.tqp[l]);
    uint64_t B = mullo64(y, D.tq[l]) - mullo64(A, P.q);
    if (B >= P.q) { B -= P.q; A += 1; }
    sumA += A;
    mw_addmul(Z, D.Mw[l], (uint32_t)B, 0, D.words);
    mw_addmul(Z, D.Mw[l], (uint32_t)(B >> 32), 1, D.words);
  }
  // W = 2 Z + q
  uint32_t W[kMaxWords], twoq[kMaxWords];
  uint64_t carry = 0, c2 = 0;
  for (int w = 0; w < kMaxWords; ++w) {
    const uint64_t z2 = ((uint64_t)Z[w] << 1) | c2;
    c2 = (uint64_t)Z[w] >> 31;
    const uint64_t cur = (z2 & 0xffffffffull) + D.qw[w] + carry;
    W[w] = (uint32_t)cur;
    carry = cur >> 32;
    const uint64_t q2 = ((uint64_t)D.qw[w] << 1);
    twoq[w] = (uint32_t)q2 | (w ? (D.qw[w - 1] >> 31) : 0u);
  }
  uint32_t rnd = 0;
  for (int l = 0; l < L; ++l) {
    if (mw_geq(W, twoq)) {
      mw_sub(W, twoq);
      rnd += 1;
    }
  }
  return (uint32_t)((sumA + rnd) % D.t);
}

// Workgroup per ciphertext: x_l = INTT(NTT(c1) NTT(s)) + c0 per limb, then the
// exact decode and the client share [m + ||q||^2]_t.
template <int LOGN>
__global__ void __launch_bounds__(NttShape<LOGN>::T)
k_decrypt(const uint64_t* __restrict__ ct, const uint64_t* __restrict__ sk_ntt,
          const uint32_t* __restrict__ qnorm2, uint32_t* __restrict__ outp, int L,
          PrimeSet ps, TwSet tws, DecodeConst D) {
  extern __shared__ uint64_t lds[];
  constexpr int N = NttShape<LOGN>::N;
  const int tid = threadIdx.x, m = blockIdx.x;
  uint64_t x[kMaxLimbs][16];
  for (int l = 0; l < L; ++l) {
    const Prime& P = ps.p[l];
    const uint64_t* c0 = ct + (((size_t)m * 2) * L + l) * N;
    const uint64_t* c1 = ct + (((size_t)m * 2 + 1) * L + l) * N;
    uint64_t v[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) v[a] = c1[coef_index<LOGN>(tid, a)];
    ntt_fwd<LOGN>(v, lds, tid, tws.tw[l], P);
#pragma unroll
    for (int a = 0; a < 16; ++a)
      v[a] = mulmod(v[a], sk_ntt[(size_t)l * N + ntt_slot<LOGN>(tid, a)], P);
    ntt_inv<LOGN>(v, lds, tid, tws.tw[l] + N, P);
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const uint64_t r = addmod(v[a], c0[coef_index<LOGN>(tid, a)], P.q);
#pragma unroll
      for (int ll = 0; ll < kMaxLimbs; ++ll)
        if (ll == l) x[ll][a] = r;
    }
  }
  const uint32_t qn = qnorm2 ? qnorm2[m] : 0u;
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    uint64_t xl[kMaxLimbs];
#pragma unroll
    for (int l = 0; l < kMaxLimbs; ++l) xl[l] = x[l][a];
    const uint32_t mm = crt_round(xl, L, ps, D);
    const uint64_t s = (uint64_t)mm + qn;
    outp[(size_t)m * N + coef_index<LOGN>(tid, a)] = (uint32_t)(s >= D.t ? s - D.t : s);
  }
}

// --------------------------------------------------------------------------
// plain form: one launch per ciphertext operation
// --------------------------------------------------------------------------

// tmp[c][l][j] = c_hat_i[c][l][j] g_hat_{i,k}[l][j]  (one query coordinate)
__global__ void __launch_bounds__(256)
k_mult_plain(const uint2* __restrict__ cq, const uint2* __restrict__ db, int i, int k,
             int d, int C, int L, int logN, PrimeSet ps, uint64_t* __restrict__ tmp) {
  const int N = 1 << logN;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 2 * L * N) return;
  const int j = g & (N - 1), l = (g >> logN) % L;
  const Prime& P = ps.p[l];
  const uint2 y = db[(((size_t)l * C + k) * d + i) * N + j];
  const uint64_t b = ((uint64_t)y.y << 27) | y.x;
  const uint2 x = cq[g];
  tmp[g] = mulmod(((uint64_t)x.y << 27) | x.x, b, P);
}

// acc[c][l][j] += tmp[c][l][j]
__global__ void __launch_bounds__(256)
k_add(uint64_t* __restrict__ acc, const uint64_t* __restrict__ tmp, int L, int logN,
      PrimeSet ps) {
  const int N = 1 << logN;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 2 * L * N) return;
  const int l = (g >> logN) % L;
  acc[g] = addmod(acc[g], tmp[g], ps.p[l].q);
}

// c0[l][j] += Delta_l [norm_j - r_j]_t   (coefficient form)
__global__ void __launch_bounds__(256)
k_add_plain(uint64_t* __restrict__ ct, const uint32_t* __restrict__ share,
            const uint32_t* __restrict__ norms, int k, int L, int logN, uint32_t t,
            PrimeSet ps) {
  const int N = 1 << logN;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= L * N) return;
  const int j = g & (N - 1), l = g >> logN;
  const Prime& P = ps.p[l];
  const uint32_t pn = norms[(size_t)k * N + j], rj = share[j];
  const uint64_t mv = pn >= rj ? pn - rj : pn + t - rj;
  ct[g] = addmod(ct[g], shoup(mv, P.delta, P.deltap, P.q), P.q);
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------

// Transform-size dispatch: every kernel built on the register NTT is
// instantiated for log2 N = 4 .. 14.
#define SANNS_LOGN_CASES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

template <int LG, typename K, typename... A>
static void ntt_launch(K kern, unsigned grid, hipStream_t st, A... args) {
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NttShape<LG>::T), NttShape<LG>::lds_bytes, st,
                     args...);
}

hipError_t launch_ntt_fwd(const uint64_t* in, uint64_t* out, int n_polys, int logN, int L,
                          const PrimeSet& ps, const TwSet& tws, uint32_t* err, int split,
                          hipStream_t st, int d, int R) {
  if (n_polys <= 0) return hipSuccess;
  if (split == 2 && (logN < 5 || d <= 0 || n_polys != R * d * L)) return hipErrorInvalidValue;
  bool pm = true;  // the matrix-core schedule's form: the short last reduction when it holds
  for (int l = 0; l < L; ++l) pm = pm && pm_delta(ps.p[l].q) != 0;
  switch (logN) {
#define SANNS_CASE(LG)                                                                    \
  case LG:                                                                                \
    if (split == 2 && pm)                                                                 \
      ntt_launch<LG>(k_ntt_fwd<LG, 2, true>, (unsigned)n_polys, st, in, out, L, ps, tws, err, \
                     d, R);                                                               \
    else if (split == 2)                                                                  \
      ntt_launch<LG>(k_ntt_fwd<LG, 2>, (unsigned)n_polys, st, in, out, L, ps, tws, err, d, R); \
    else if (split == 1)                                                                  \
      ntt_launch<LG>(k_ntt_fwd<LG, 1>, (unsigned)n_polys, st, in, out, L, ps, tws, err, d, R); \
    else                                                                                  \
      ntt_launch<LG>(k_ntt_fwd<LG, 0>, (unsigned)n_polys, st, in, out, L, ps, tws, err, d, R); \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ntt_inv(uint64_t* io, int n_polys, int logN, int L, const PrimeSet& ps,
                          const TwSet& tws, hipStream_t st) {
  if (n_polys <= 0) return hipSuccess;
  switch (logN) {
#define SANNS_CASE(LG)                                                 \
  case LG:                                                             \
    ntt_launch<LG>(k_ntt_inv<LG>, (unsigned)n_polys, st, io, L, ps, tws); \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_masks(const MaskKey& K, const uint64_t* qids, const uint32_t* work, int C,
                        int M, int logN, uint32_t t, uint64_t tone, uint32_t* share,
                        hipStream_t st) {
  const long total = (long)M * ((1 << logN) >> 2);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_masks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, K,
                     qids, work, C, M, 1 << logN, t, tone, share);
  return hipGetLastError();
}

hipError_t launch_intt_mask(uint64_t* ct, const uint32_t* share, const uint32_t* norms,
                            const uint32_t* work, int C, int M, int logN, int L, uint32_t t,
                            const PrimeSet& ps, const TwSet& tws, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const int n = M * 2 * L, Qa = work ? 0 : M / C;
  const unsigned grid = (unsigned)((n + 7) / 8 * 8);
  switch (logN) {
#define SANNS_CASE(LG)                                                                  \
  case LG:                                                                              \
    ntt_launch<LG>(k_intt_mask<LG>, grid, st, ct, share, norms, work, C, L, t, ps, tws, \
                   n, Qa);                                                              \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int QT, int CT>
static hipError_t launch_mac_t(const uint2* qntt, const uint2* db, const void* tiles,
                               int n_tiles, int Q, int d, int L, int logN, int C,
                               const PrimeSet& ps, uint64_t* out, hipStream_t st) {
  const int N = 1 << logN;
  const int bs = N < 256 ? N : 256;
  const long nb = (long)(N / bs) * n_tiles * L;
  const long per_xcd = (nb + 7) >> 3;
  if (tiles)
    hipLaunchKernelGGL((k_mac<QT, CT, false>), dim3((unsigned)(per_xcd * 8)), dim3(bs), 0, st,
                       qntt, db, (const MacTile<QT, CT>*)tiles, n_tiles, Q, d, L, logN, C,
                       (int)nb, ps, out);
  else
    hipLaunchKernelGGL((k_mac<QT, CT, true>), dim3((unsigned)(per_xcd * 8)), dim3(bs), 0, st,
                       qntt, db, (const MacTile<QT, CT>*)tiles, n_tiles, Q, d, L, logN, C,
                       (int)nb, ps, out);
  return hipGetLastError();
}

size_t mac_tile_bytes(int QT, int CT) {
#define SANNS_MAC_SIZE(a, b) \
  if (QT == a && CT == b) return sizeof(MacTile<a, b>);
  SANNS_MAC_SHAPES(SANNS_MAC_SIZE)
#undef SANNS_MAC_SIZE
  return 0;
}

hipError_t launch_mac(int QT, int CT, const uint2* qntt, const uint2* db, const void* tiles,
                      int n_tiles, int Q, int d, int L, int logN, int C, const PrimeSet& ps,
                      uint64_t* out, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
#define SANNS_MAC_CASE(a, b) \
  if (QT == a && CT == b)    \
    return launch_mac_t<a, b>(qntt, db, tiles, n_tiles, Q, d, L, logN, C, ps, out, st);
  SANNS_MAC_SHAPES(SANNS_MAC_CASE)
#undef SANNS_MAC_CASE
  return hipErrorInvalidValue;
}

template <int QT, int CT, int QG, int CG, int S, int DI, int UNR>
static hipError_t launch_mac_lds_t(const uint2* qntt, const uint2* db, int Q, int d, int L,
                                   int logN, int C, const PrimeSet& ps, uint64_t* out,
                                   hipStream_t st) {
  constexpr int QB = QT * QG, CB = CT * CG;
  const int N = 1 << logN;
  if (N % S) return hipErrorInvalidValue;
  const long nb = (long)(N / S) * L * ((Q + QB - 1) / QB) * ((C + CB - 1) / CB);
  if (nb > 0x7fffffffL) return hipErrorInvalidValue;
  const int per_xcd = (int)((nb + 7) / 8);
  if (d > (255 / DI) * DI)
    hipLaunchKernelGGL((k_mac_lds<QT, CT, QG, CG, S, DI, UNR, true>), dim3(per_xcd * 8),
                       dim3(S * QG * CG), 0, st, qntt, db, Q, d, L, logN, C, (int)nb, ps, out);
  else
    hipLaunchKernelGGL((k_mac_lds<QT, CT, QG, CG, S, DI, UNR, false>), dim3(per_xcd * 8),
                       dim3(S * QG * CG), 0, st, qntt, db, Q, d, L, logN, C, (int)nb, ps, out);
  return hipGetLastError();
}

template <int QT, int CT, int QG, int CG, int S, int DI, int UNR>
static hipError_t launch_mac_dl_t(const uint2* qntt, const uint2* db, int Q, int d, int L,
                                  int logN, int C, const PrimeSet& ps, uint64_t* out,
                                  hipStream_t st) {
  constexpr int QB = QT * QG, CB = CT * CG;
  const int N = 1 << logN;
  if (N % S) return hipErrorInvalidValue;
  const long nb = (long)(N / S) * L * ((Q + QB - 1) / QB) * ((C + CB - 1) / CB);
  if (nb > 0x7fffffffL) return hipErrorInvalidValue;
  const int per_xcd = (int)((nb + 7) / 8);
  if (d > (255 / DI) * DI)
    hipLaunchKernelGGL((k_mac_dl<QT, CT, QG, CG, S, DI, UNR, true>), dim3(per_xcd * 8),
                       dim3(S * QG * CG), 0, st, qntt, db, Q, d, L, logN, C, (int)nb, ps, out);
  else
    hipLaunchKernelGGL((k_mac_dl<QT, CT, QG, CG, S, DI, UNR, false>), dim3(per_xcd * 8),
                       dim3(S * QG * CG), 0, st, qntt, db, Q, d, L, logN, C, (int)nb, ps, out);
  return hipGetLastError();
}

hipError_t launch_mac_lds(int variant, const uint2* qntt, const uint2* db, int Q, int d, int L,
                          int logN, int C, const PrimeSet& ps, uint64_t* out, hipStream_t st) {
  switch (variant) {
#define SANNS_LDS_CASE(id, qt, ct, qg, cg, s, di, unr) \
  case id:                                             \
    return launch_mac_lds_t<qt, ct, qg, cg, s, di, unr>(qntt, db, Q, d, L, logN, C, ps, out, st);
    SANNS_MAC_LDS_VARIANTS(SANNS_LDS_CASE)
#undef SANNS_LDS_CASE
#define SANNS_DL_CASE(id, qt, ct, qg, cg, s, di, unr) \
  case id:                                            \
    return launch_mac_dl_t<qt, ct, qg, cg, s, di, unr>(qntt, db, Q, d, L, logN, C, ps, out, st);
    SANNS_MAC_DL_VARIANTS(SANNS_DL_CASE)
#undef SANNS_DL_CASE
    default:
      return hipErrorInvalidValue;
  }
}

int mac_lds_min_n(int variant) {
  switch (variant) {
#define SANNS_LDS_S(id, qt, ct, qg, cg, s, di, unr) \
  case id:                                     \
    return s;
    SANNS_MAC_LDS_VARIANTS(SANNS_LDS_S)
    SANNS_MAC_DL_VARIANTS(SANNS_LDS_S)
#undef SANNS_LDS_S
    default:
      return 0;
  }
}

int persistent_logn(int shape) {
  switch (shape) {
#define SANNS_PS_LOGN(id, lg, qt, ct, qg, cg, di) \
  case id:                                       \
    return lg;
    SANNS_PERSIST_SHAPES(SANNS_PS_LOGN)
#undef SANNS_PS_LOGN
    default:
      return 0;
  }
}

int persistent_max_d(int shape) {
  switch (shape) {
#define SANNS_PS_MAXD(id, lg, qt, ct, qg, cg, di) \
  case id:                                       \
    return (255 / di) * di;
    SANNS_PERSIST_SHAPES(SANNS_PS_MAXD)
#undef SANNS_PS_MAXD
    default:
      return 0;
  }
}

int persistent_default_shape(int logN) {
  switch (logN) {
    case 11: return 61;
    case 12: return 51;
    case 13: return 41;
    case 14: return 71;
    default: return 0;
  }
}

template <int LOGN, int QT, int CT, int QG, int CG, int DI>
static hipError_t launch_persistent_t(const PersistArgs& A, const PrimeSet& ps,
                                      const TwSet& tws, hipStream_t st) {
  constexpr int T = NttShape<LOGN>::T, S = T / (QG * CG);
  constexpr size_t lds_mac = MacDlShape<QT, CT, QG, CG, S, DI>::lds_bytes;
  constexpr size_t lds = lds_mac > NttShape<LOGN>::lds_bytes ? lds_mac : NttShape<LOGN>::lds_bytes;
  auto kern = k_persistent<LOGN, QT, CT, QG, CG, DI, kPersistTileQ, kPersistTileC>;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, T, lds);
  if (e != hipSuccess) return e;
  long items = (long)A.Q * A.d * 2 * A.L + A.M;
  long blocks = (long)cus * (per_cu > 0 ? per_cu : 1);
  if (blocks > items) blocks = items;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, A.ctrl, kPersistCtrlWords, 0u);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(T), lds, st, A, ps, tws);
  return hipGetLastError();
}

hipError_t launch_persistent(int shape, const PersistArgs& A, const PrimeSet& ps,
                             const TwSet& tws, hipStream_t st) {
  switch (shape) {
#define SANNS_PS_CASE(id, lg, qt, ct, qg, cg, di) \
  case id:                                       \
    return launch_persistent_t<lg, qt, ct, qg, cg, di>(A, ps, tws, st);
    SANNS_PERSIST_SHAPES(SANNS_PS_CASE)
#undef SANNS_PS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_gather(const void* pts, int is_signed, long n, int d,
                         const int64_t* slot_point, long base, long total, int logN,
                         int16_t* gt, uint32_t* norms, uint32_t* err, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     (const uint8_t*)pts, is_signed, n, d, slot_point, base, total, logN, gt,
                     norms, err);
  return hipGetLastError();
}

template <typename G>
static hipError_t launch_encode_ntt_t(const G* gt, uint2* dbres, int k0, int nk, int C, int d,
                                      int logN, int L, const PrimeSet& ps, const TwSet& tws,
                                      hipStream_t st) {
  const unsigned grid = (unsigned)((long)L * nk * d);
  if (grid == 0) return hipSuccess;
  switch (logN) {
#define SANNS_CASE(LG)                                                                     \
  case LG:                                                                                 \
    ntt_launch<LG>(k_encode_ntt<LG, G>, grid, st, gt, dbres, k0, nk, C, d, L, ps, tws);     \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_encode_ntt(const int16_t* gt, uint2* dbres, int k0, int nk, int C, int d,
                             int logN, int L, const PrimeSet& ps, const TwSet& tws,
                             hipStream_t st) {
  return launch_encode_ntt_t(gt, dbres, k0, nk, C, d, logN, L, ps, tws, st);
}

hipError_t launch_encode_ntt32(const int32_t* gt, uint2* dbres, int k0, int nk, int C, int d,
                               int logN, int L, const PrimeSet& ps, const TwSet& tws,
                               hipStream_t st) {
  return launch_encode_ntt_t(gt, dbres, k0, nk, C, d, logN, L, ps, tws, st);
}

// Block per range r: slot[off[r] + i] = start[r] + i for i < len[r] (writes
// past `total` are dropped); launched after slot has been filled with -1.
__global__ void __launch_bounds__(256)
k_slot_ranges(const int64_t* __restrict__ start, const int64_t* __restrict__ len,
              const int64_t* __restrict__ off, int64_t* __restrict__ slot, long total) {
  const int r = blockIdx.x;
  const long s0 = start[r], n = len[r], o = off[r];
  for (long i = threadIdx.x; i < n; i += blockDim.x)
    if (o + i >= 0 && o + i < total) slot[o + i] = s0 + i;
}

__global__ void __launch_bounds__(256) k_fill_i64(int64_t* __restrict__ p, long n, int64_t v) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) p[g] = v;
}

hipError_t launch_slot_ranges(const int64_t* start, const int64_t* len, const int64_t* off,
                              int R, int64_t* slot, long total, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, slot,
                     total, (int64_t)-1);
  if (R > 0)
    hipLaunchKernelGGL(k_slot_ranges, dim3((unsigned)R), dim3(256), 0, st, start, len, off, slot,
                       total);
  return hipGetLastError();
}

hipError_t launch_gather32(const void* pts, int kind, long n, int d, const uint32_t* norm_shares,
                           uint32_t t, const int64_t* slot_point, long base, long total,
                           int logN, int32_t* gt, uint32_t* norms, uint32_t* err,
                           hipStream_t st) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather32, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, pts,
                     kind, n, d, norm_shares, t, slot_point, base, total, logN, gt, norms, err);
  return hipGetLastError();
}

hipError_t launch_sk_ntt(const int8_t* sk, uint64_t* out, int logN, int L, const PrimeSet& ps,
                         const TwSet& tws, hipStream_t st) {
  switch (logN) {
#define SANNS_CASE(LG)                                                   \
  case LG:                                                               \
    ntt_launch<LG>(k_sk_ntt<LG>, (unsigned)L, st, sk, out, ps, tws);     \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rerand(const MaskKey& K, const uint64_t* qids, const uint32_t* work, int C,
                         int M, int L, int logN, const uint64_t* pk_ntt, uint64_t* ct,
                         const PrimeSet& ps, const TwSet& tws, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  switch (logN) {
#define SANNS_CASE(LG)                                                                    \
  case LG:                                                                                \
    ntt_launch<LG>(k_rerand<LG>, (unsigned)(M * L), st, K, qids, work, C, L, pk_ntt, ct, ps, \
                   tws);                                                                  \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_intt_mask_cp(uint64_t* ct, const uint32_t* share, const uint32_t* norms,
                               const uint32_t* work, int C, int M, int logN, int L, uint32_t t,
                               const MaskKey& K, const uint64_t* qids, const CpConst& cp,
                               const DigitSet& ds, const PrimeSet& ps, const TwSet& tws,
                               uint64_t* flood, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const int N = 1 << logN;
  const long nf = (long)M * (N / 2);
  int8_t* errs = reinterpret_cast<int8_t*>(flood + (size_t)M * L * N);
  const int n = M * 2 * L, Qa = work ? 0 : M / C;
  const unsigned grid = (unsigned)((n + 7) / 8 * 8);
  hipLaunchKernelGGL(k_cp_noise, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, K, qids,
                     work, C, (long)M, N, L, cp, ds, ps, flood, errs);
  switch (logN) {
#define SANNS_CASE(LG)                                                                       \
  case LG:                                                                                   \
    ntt_launch<LG>(k_intt_mask_cp<LG>, grid, st, ct, share, norms, work, C, L, t,            \
                   (const uint64_t*)flood, (const int8_t*)errs, ps, tws, n, Qa);              \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_keygen(uint64_t seed, int N, int8_t* sk, hipStream_t st) {
  const int nb = N / 8;
  hipLaunchKernelGGL(k_keygen, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, seed, N, sk);
  return hipGetLastError();
}

hipError_t launch_sample_enc(uint64_t seed, uint32_t purpose_a, uint32_t purpose_e, int Qd,
                             int d, int L, int N, const PrimeSet& ps, uint64_t* a, int16_t* e,
                             hipStream_t st) {
  if (Qd <= 0) return hipSuccess;
  const long ta = (long)Qd * L * (N / 4), te = (long)Qd * (N / 8);
  hipLaunchKernelGGL(k_sample_a, dim3((unsigned)((ta + 255) / 256)), dim3(256), 0, st, seed,
                     purpose_a, d, L, N, ta, ps, a);
  hipLaunchKernelGGL(k_sample_e, dim3((unsigned)((te + 255) / 256)), dim3(256), 0, st, seed,
                     purpose_e, d, N, te, e);
  return hipGetLastError();
}

hipError_t launch_encrypt(const uint64_t* a, const int16_t* e, const int32_t* msgs,
                          const uint64_t* sk_ntt, uint64_t* ct, int Qd, int L, int logN,
                          uint32_t t, const PrimeSet& ps, const TwSet& tws, hipStream_t st) {
  if (Qd <= 0) return hipSuccess;
  switch (logN) {
#define SANNS_CASE(LG)                                                                 \
  case LG:                                                                             \
    ntt_launch<LG>(k_encrypt<LG>, (unsigned)(Qd * L), st, a, e, msgs, sk_ntt, ct, L, t, \
                   ps, tws);                                                           \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_decrypt(const uint64_t* ct, int M, const uint64_t* sk_ntt,
                          const uint32_t* qnorm2, uint32_t* out, int L, int logN,
                          const PrimeSet& ps, const TwSet& tws, const DecodeConst& D,
                          hipStream_t st) {
  if (M <= 0) return hipSuccess;
  switch (logN) {
#define SANNS_CASE(LG)                                                                   \
  case LG:                                                                               \
    ntt_launch<LG>(k_decrypt<LG>, (unsigned)M, st, ct, sk_ntt, qnorm2, out, L, ps, tws, D); \
    break;
    SANNS_LOGN_CASES(SANNS_CASE)
#undef SANNS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mult_plain(const uint2* cq, const uint2* db, int i, int k, int d, int C,
                             int L, int logN, const PrimeSet& ps, uint64_t* tmp,
                             hipStream_t st) {
  const int total = 2 * L * (1 << logN);
  hipLaunchKernelGGL(k_mult_plain, dim3((total + 255) / 256), dim3(256), 0, st, cq, db, i, k,
                     d, C, L, logN, ps, tmp);
  return hipGetLastError();
}

hipError_t launch_add(uint64_t* acc, const uint64_t* tmp, int L, int logN, const PrimeSet& ps,
                      hipStream_t st) {
  const int total = 2 * L * (1 << logN);
  hipLaunchKernelGGL(k_add, dim3((total + 255) / 256), dim3(256), 0, st, acc, tmp, L, logN,
                     ps);
  return hipGetLastError();
}

hipError_t launch_add_plain(uint64_t* ct, const uint32_t* share, const uint32_t* norms, int k,
                            int L, int logN, uint32_t t, const PrimeSet& ps, hipStream_t st) {
  const int total = L * (1 << logN);
  hipLaunchKernelGGL(k_add_plain, dim3((total + 255) / 256), dim3(256), 0, st, ct, share,
                     norms, k, L, logN, t, ps);
  return hipGetLastError();
}

}  // namespace sanns
