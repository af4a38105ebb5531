// Matrix-core schedule of the all-pairs multiply-accumulate (gfx950 int8 MFMA).
//
// For one NTT slot p of limb l, the multiply-accumulate of a batch (Section
// 4.2: every query ciphertext against every chunk) is an exact integer matrix
// product with rows r = (query q, component c), columns chunks k and the
// contraction over the d coordinates:
//     acc[r][k] = sum_i c_hat[q][i][c][p] * g_hat[k][i][p]      (mod q_l).
// Both operands are residues below 2^54.  Each is written with seven signed
// base-256 digits  x = sum_a x_a 256^a,  x_a in [-128, 127]  (x_6 in [0, 64]),
// obtained from the bytes of x + B, B = sum_a 128 256^a:  x_a = byte_a(x + B)
// - 128, i.e. the byte XOR 0x80 read as int8.  Then
//     sum_i x y = sum_{s=0}^{12} 256^s S_s,   S_s = sum_{a+b=s} sum_i x_a[i] y_b[i],
// where every S_s is an exact int32 sum of int8 products (|S_s| < 7 2^14 Dp),
// which is what the int8 MFMA computes: 49 digit-pair products per residue
// pair, 13 accumulators per output.  The S_s are folded into a residue in
// [0, q_l) with 64-bit integer steps and Shoup products.  Nothing here is
// approximate: the result equals the one of the 64-bit vector kernels.
//
// Layouts (Dp = d rounded up to a multiple of 64, the coordinates of one MFMA
// step being 64s .. 64s + 63; coordinate i >= d holds the digit 0):
//   query digits    [L][N][R][7][Dp] int8    R = 2Q rows, row = 2q + c
//   database digits [L][N][C][Sk] int8       Sk = 7 Dp + 16: digit rows, then
//                                            16 bytes of padding (LDS banks)
//   slot-major sums [L][N][R][C] uint64 in [0, q_l)
// Fragment of one lane (row or column m = lane % 16, group g = lane / 16) at
// step s: the 16 bytes of one digit row at coordinates 64s + 16g .. + 15.
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "launch.h"

namespace sanns {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr uint64_t kDigitBias = 0x0080808080808080ull;  // 128 in each of bytes 0..6
constexpr int kMfmaRows = 64;    // rows per workgroup: 4 waves x 16
constexpr int kMfmaChunks = 32;  // chunks per workgroup: 2 MFMA column tiles
constexpr int kMfmaSlots = 8;    // consecutive slots per workgroup
constexpr int kDigitSlots = 32;  // slots per workgroup of the digit transposes

// The signed digits of x < 2^54 as the bytes of a word (byte 7 is zero).
__device__ __forceinline__ uint64_t digit_word(uint64_t x) {
  return (x + kDigitBias) ^ kDigitBias;
}

// Byte `a` of each of four words, packed low to high.
__device__ __forceinline__ uint32_t gather_byte(uint64_t y0, uint64_t y1, uint64_t y2,
                                                uint64_t y3, int a) {
  const int sh = 8 * a;
  return (uint32_t)((y0 >> sh) & 0xff) | (uint32_t)(((y1 >> sh) & 0xff) << 8) |
         (uint32_t)(((y2 >> sh) & 0xff) << 16) | (uint32_t)(((y3 >> sh) & 0xff) << 24);
}

// Transpose-and-digitise: a workgroup takes kDigitSlots consecutive slots of
// one (limb, entity) pair, where the entity is a query row (source: the
// query NTT form [Q][d][2][L][N] uint64) or a database chunk (source: the
// database residues [L][C][d][N] as 27-bit halves), stages the d x 32 words in
// LDS, and writes each slot's 7 digit rows of Dp bytes (16 bytes per store,
// zero digits past coordinate d).
template <bool DB>
__global__ void __launch_bounds__(256)
k_to_digits(const void* __restrict__ src, int8_t* __restrict__ dst, int n_ent, int d, int Dp,
            int L, int logN, int C, int Sk) {
  extern __shared__ uint64_t lw[];  // [Dp][kDigitSlots + 1]
  constexpr int P1 = kDigitSlots + 1;
  const int N = 1 << logN;
  const int groups = N / kDigitSlots;
  int b = blockIdx.x;
  const int pg = b % groups;
  b /= groups;
  const int ent = b % n_ent, l = b / n_ent;
  const int p0 = pg * kDigitSlots;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < Dp * kDigitSlots; idx += 256) {
    const int i = idx / kDigitSlots, pp = idx % kDigitSlots;
    uint64_t x = 0;
    if (i < d) {
      if (DB) {
        const uint2 h = reinterpret_cast<const uint2*>(
            src)[(((size_t)l * C + ent) * d + i) * N + p0 + pp];
        x = (uint64_t)h.x + ((uint64_t)h.y << 27);
      } else {
        const int q = ent >> 1, c = ent & 1;
        x = reinterpret_cast<const uint64_t*>(
            src)[((((size_t)q * d + i) * 2 + c) * L + l) * N + p0 + pp];
      }
    }
    lw[i * P1 + pp] = digit_word(x);
  }
  __syncthreads();
  const int cg_n = Dp / 16;
  for (int u = tid; u < kDigitSlots * cg_n; u += 256) {
    const int cg = u % cg_n, pp = u / cg_n;
    const int p = p0 + pp;
    uint64_t y[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = lw[(16 * cg + j) * P1 + pp];
    int8_t* row = DB ? dst + (((size_t)l * N + p) * C + ent) * Sk
                     : dst + (((size_t)l * N + p) * n_ent + ent) * (size_t)(7 * Dp);
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      uint4 v;
      v.x = gather_byte(y[0], y[1], y[2], y[3], a);
      v.y = gather_byte(y[4], y[5], y[6], y[7], a);
      v.z = gather_byte(y[8], y[9], y[10], y[11], a);
      v.w = gather_byte(y[12], y[13], y[14], y[15], a);
      *reinterpret_cast<uint4*>(row + a * Dp + 16 * cg) = v;
    }
    if (DB && cg == 0) *reinterpret_cast<uint4*>(row + 7 * Dp) = make_uint4(0, 0, 0, 0);
  }
}

__device__ __forceinline__ int32_t opaque_i32(int32_t x) {
  asm("" : "+v"(x));
  return x;
}

// Residue in [0, q) of V = sum_s S_s 256^s (Dp <= 256, so |S_s| < 2^29):
//   g0 = S0 + S1 2^8 + S2 2^16 + S3 2^24          |g0| < 2^53
//   g1 = S4 + ... + S7 2^24  (weight 2^32)        |g1| < 2^53
//   h  = S8 + ... + S11 2^24 + S12 2^32  (weight 2^64),  |h| < 2^57
// and V = g0 + g1 2^32 + h 2^64.
__device__ __forceinline__ uint64_t fold_digit_sums(const int32_t (&S)[13], const Prime& P,
                                                    const DigitConst& D, uint64_t nq) {
  const int32_t k8 = opaque_i32(1 << 8), k16 = opaque_i32(1 << 16), k24 = opaque_i32(1 << 24);
  auto group = [&](int s) {
    int64_t g = (int64_t)S[s];
    g += (int64_t)S[s + 1] * k8;
    g += (int64_t)S[s + 2] * k16;
    g += (int64_t)S[s + 3] * k24;
    return g;
  };
  const int64_t g0 = group(0), g1 = group(4);
  const int64_t h = group(8) + (int64_t)((uint64_t)(uint32_t)S[12] << 32);
  const uint64_t x0 = (uint64_t)(g0 + (int64_t)D.offa);
  const uint64_t x1 = (uint64_t)(g1 + (int64_t)D.offa);
  const uint64_t x2 = (uint64_t)(h + (int64_t)D.offb);
  const uint64_t s = x0 + shoup_approx(x1, D.w32, D.w32p, nq) +
                     shoup_approx(x2, D.w64, D.w64p, nq);  // < 2^55 + 8q < 2^58
  const uint64_t r = shoup_approx(s, 1, P.one, nq);       // [0, 4q)
  return csub(csub(r, 2 * P.q), P.q);
}

// One workgroup: 64 rows x 32 chunks of kMfmaSlots consecutive slots of one
// limb.  Wave w owns rows 16w .. 16w + 15 of the tile and both 16-chunk
// column tiles; its query fragments come straight from global memory, the
// chunk tile's database digits are staged in LDS (global_load_lds, double
// buffered across slots).  Workgroups are numbered so that the tiles of one
// slot range run back to back on one XCD, which shares the operands in its L2.
template <int NKS>
__global__ void __launch_bounds__(256, 2)
k_mac_mfma(const int8_t* __restrict__ qd, const int8_t* __restrict__ dbd, int R, int C, int L,
           int logN, int n_items, PrimeSet ps, DigitSet ds, uint64_t* __restrict__ sums) {
  constexpr int Dp = 64 * NKS, Sk = 7 * Dp + 16;
  constexpr int BU = kMfmaChunks * Sk / 16;  // 16-byte units of one staged tile
  constexpr int BR = (BU + 255) / 256;
  __shared__ uint4 sb0[BU], sb1[BU];
  const int N = 1 << logN;
  const int per_xcd = (n_items + 7) >> 3;
  const int lin = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lin >= n_items) return;
  const int nrt = (R + kMfmaRows - 1) / kMfmaRows, nct = (C + kMfmaChunks - 1) / kMfmaChunks;
  const int tile = lin % (nrt * nct), sg = lin / (nrt * nct);
  const int rt = tile % nrt, ctile = tile / nrt;
  const int l = sg % L, p0 = (sg / L) * kMfmaSlots;
  const int k0 = ctile * kMfmaChunks;
  const int nk = C - k0 < kMfmaChunks ? C - k0 : kMfmaChunks;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int m16 = lane & 15, g = lane >> 4;
  const int wrow0 = rt * kMfmaRows + 16 * w;
  const bool idle = wrow0 >= R;  // uniform over the wave
  const int arow = wrow0 + m16 < R ? wrow0 + m16 : R - 1;
  const Prime& P = ps.p[l];
  const DigitConst& D = ds.c[l];
  const uint64_t nq = 0 - P.q;
  const int bunits = nk * Sk / 16;

  auto stage = [&](int p, uint4* buf) {
    const uint4* src =
        reinterpret_cast<const uint4*>(dbd + (((size_t)l * N + p) * C + k0) * Sk);
#pragma unroll
    for (int m = 0; m < BR; ++m) {
      const int u = tid + 256 * m;
      if (u < bunits)
        __builtin_amdgcn_global_load_lds(
            (const void*)(src + u),
            (__attribute__((address_space(3))) void*)(buf + 256 * m + 64 * w), 16, 0, 0);
    }
  };

  stage(p0, sb0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int jj = 0; jj < kMfmaSlots; ++jj) {
    const int p = p0 + jj;
    const uint4* cur = (jj & 1) ? sb1 : sb0;
    if (jj + 1 < kMfmaSlots) stage(p + 1, (jj & 1) ? sb0 : sb1);
    if (!idle) {
      v4i acc[2][13];
      const int8_t* abase = qd + (((size_t)l * N + p) * R + arow) * (size_t)(7 * Dp) + 16 * g;
      const int8_t* bbase = reinterpret_cast<const int8_t*>(cur) + m16 * Sk + 16 * g;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        v4i af[7];
#pragma unroll
        for (int a = 0; a < 7; ++a)
          af[a] = *reinterpret_cast<const v4i*>(abase + a * Dp + 64 * ks);
#pragma unroll
        for (int b = 0; b < 7; ++b)
#pragma unroll
          for (int cs = 0; cs < 2; ++cs) {
            const v4i bf =
                *reinterpret_cast<const v4i*>(bbase + cs * 16 * Sk + b * Dp + 64 * ks);
            // the first product of diagonal a + b starts from a zero
            // accumulator (b = 0, or a = 6 for the diagonals above 6)
#pragma unroll
            for (int a = 0; a < 7; ++a)
              acc[cs][a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                  af[a], bf, (ks == 0 && (b == 0 || a == 6)) ? v4i{0, 0, 0, 0} : acc[cs][a + b],
                  0, 0, 0);
          }
      }
      // lane holds rows 4g .. 4g + 3 of the wave's 16, chunk m16 of each column tile
#pragma unroll
      for (int cs = 0; cs < 2; ++cs) {
        const int kk = cs * 16 + m16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int32_t S[13];
#pragma unroll
          for (int s = 0; s < 13; ++s) S[s] = acc[cs][s][e];
          const uint64_t v = fold_digit_sums(S, P, D, nq);
          const int row = wrow0 + 4 * g + e;
          if (row < R && kk < nk) sums[(((size_t)l * N + p) * R + row) * C + k0 + kk] = v;
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// Slot-major sums [L][N][R][C] -> ciphertexts [Q C][2][L][N] (output m = q C + k,
// component c = row & 1): 64 slots x 32 chunks of one row per workgroup.
__global__ void __launch_bounds__(256)
k_sums_to_ct(const uint64_t* __restrict__ sums, uint64_t* __restrict__ ct, int R, int C, int L,
             int logN) {
  __shared__ uint64_t t[32][65];
  const int N = 1 << logN;
  const int ng = N / 64, nkg = (C + 31) / 32;
  int b = blockIdx.x;
  const int kg = b % nkg;
  b /= nkg;
  const int row = b % R;
  b /= R;
  const int pg = b % ng, l = b / ng;
  const int p0 = pg * 64, k0 = kg * 32;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 64 * 32; idx += 256) {
    const int kk = idx % 32, pp = idx / 32;
    if (k0 + kk < C) t[kk][pp] = sums[(((size_t)l * N + p0 + pp) * R + row) * C + k0 + kk];
  }
  __syncthreads();
  const int q = row >> 1, c = row & 1;
  for (int idx = tid; idx < 64 * 32; idx += 256) {
    const int pp = idx % 64, kk = idx / 64;
    if (k0 + kk < C)
      ct[((((size_t)q * C + k0 + kk) * 2 + c) * L + l) * N + p0 + pp] = t[kk][pp];
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

int mfma_padded_d(int d) { return (d + 63) / 64 * 64; }
int mfma_db_stride(int d) { return 7 * mfma_padded_d(d) + 16; }

bool mfma_supported(int logN, int d) {
  return logN >= 6 && d >= 1 && d <= kMfmaMaxD;
}

hipError_t launch_query_digits(const uint64_t* qntt, int8_t* qd, int Q, int d, int L, int logN,
                               hipStream_t st) {
  const int Dp = mfma_padded_d(d), N = 1 << logN;
  const long nb = (long)L * 2 * Q * (N / kDigitSlots);
  if (nb <= 0) return hipSuccess;
  const size_t lds = (size_t)Dp * (kDigitSlots + 1) * sizeof(uint64_t);
  hipLaunchKernelGGL(k_to_digits<false>, dim3((unsigned)nb), dim3(256), lds, st,
                     (const void*)qntt, qd, 2 * Q, d, Dp, L, logN, 0, 0);
  return hipGetLastError();
}

hipError_t launch_db_digits(const uint2* dbres, int8_t* dbd, int C, int d, int L, int logN,
                            hipStream_t st) {
  const int Dp = mfma_padded_d(d), N = 1 << logN;
  const long nb = (long)L * C * (N / kDigitSlots);
  if (nb <= 0) return hipSuccess;
  const size_t lds = (size_t)Dp * (kDigitSlots + 1) * sizeof(uint64_t);
  hipLaunchKernelGGL(k_to_digits<true>, dim3((unsigned)nb), dim3(256), lds, st,
                     (const void*)dbres, dbd, C, d, Dp, L, logN, C, mfma_db_stride(d));
  return hipGetLastError();
}

template <int NKS>
static void launch_mac_mfma_t(const int8_t* qd, const int8_t* dbd, int R, int C, int L, int logN,
                              const PrimeSet& ps, const DigitSet& ds, uint64_t* sums,
                              hipStream_t st) {
  const int N = 1 << logN;
  const long n_items = (long)L * (N / kMfmaSlots) * ((R + kMfmaRows - 1) / kMfmaRows) *
                       ((C + kMfmaChunks - 1) / kMfmaChunks);
  const long per_xcd = (n_items + 7) >> 3;
  hipLaunchKernelGGL(k_mac_mfma<NKS>, dim3((unsigned)(per_xcd * 8)), dim3(256), 0, st, qd, dbd,
                     R, C, L, logN, (int)n_items, ps, ds, sums);
}

hipError_t launch_mac_mfma(const int8_t* qd, const int8_t* dbd, int Q, int d, int C, int L,
                           int logN, const PrimeSet& ps, const DigitSet& ds, uint64_t* sums,
                           uint64_t* ct_out, hipStream_t st) {
  if (!mfma_supported(logN, d)) return hipErrorInvalidValue;
  if (Q <= 0 || C <= 0) return hipSuccess;
  const int R = 2 * Q;
  switch (mfma_padded_d(d) / 64) {
    case 1: launch_mac_mfma_t<1>(qd, dbd, R, C, L, logN, ps, ds, sums, st); break;
    case 2: launch_mac_mfma_t<2>(qd, dbd, R, C, L, logN, ps, ds, sums, st); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int N = 1 << logN;
  const long nb = (long)L * (N / 64) * R * ((C + 31) / 32);
  hipLaunchKernelGGL(k_sums_to_ct, dim3((unsigned)nb), dim3(256), 0, st, sums, ct_out, R, C, L,
                     logN);
  return hipGetLastError();
}

}  // namespace sanns
