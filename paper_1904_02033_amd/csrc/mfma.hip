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
// pair, 13 accumulators per output.  The S_s are folded into a value below
// 2^58 congruent to the sum (signed 32 x 32 -> 64-bit multiply-adds, and
// either 2^54 = delta (mod q_l) when q_l = 2^54 - delta with a small delta, or
// Shoup products), which the sums transpose reduces to [0, q_l).  Nothing here
// is approximate: the result equals the one of the 64-bit vector kernels.
//
// Layouts (Dp = d rounded up to a multiple of 32, Dq = d rounded up to a
// multiple of 64; the contraction runs in steps of 64 coordinates and, when
// Dp is an odd multiple of 32, a last step of 32; coordinate i >= d holds the
// digit 0):
//   query digits    [L][N][R][7][Dq] int8    R = 2Q rows, row = 2q + c (rows
//                                            of whole 128-byte lines)
//   database digits [L][N][C][Sk] int8       Sk = 7 Dp + 16: digit rows, then
//                                            16 bytes of padding (LDS banks)
//   slot-major sums [L][N][Rp][Cp] uint64 below 2^58, congruent mod q_l (R and
//                   C padded to whole tiles of 64 rows and 64 chunks)
// Fragment of one lane (row or column m = lane % 16, group g = lane / 16) at
// step s: the 16 bytes of one digit row at coordinates 64s + 16g .. + 15, or
// in a 32-coordinate step the 8 bytes at 64s + 8g .. + 7.
#include <hip/hip_runtime.h>
#include <type_traits>
#include "kernels.h"
#include "launch.h"
#include "chacha.h"

namespace sanns {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr uint64_t kDigitBias = 0x0080808080808080ull;  // 128 in each of bytes 0..6
constexpr int kMfmaRows = 64;    // rows per workgroup: 4 waves x 16
constexpr int kMfmaChunks = 64;  // chunks per workgroup: 4 stages of one 16-chunk MFMA column tile
constexpr int kMfmaSlots = 8;    // consecutive slots per workgroup
constexpr int kDigitGroup = 32;  // slots per group of the query NTT form (form 2)
constexpr int kQueryDigitSlots = 16;  // slots per workgroup of the query digit transpose
// The database digit region ends with this many spare bytes: a staged column
// tile may run past the last chunk (k_mac_mfma checks the bound at compile
// time).
constexpr size_t kMfmaDbSlack = 64 * 1024;
// s_waitcnt immediates (gfx9 encoding): vmcnt <= n (bits 3:0 and 15:14),
// expcnt and lgkmcnt not waited for (7 in bits 6:4, 15 in bits 11:8).
constexpr int vmcnt_wait(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int kWaitAllVmem = vmcnt_wait(0);
constexpr int kWaitAllBut7Vmem = vmcnt_wait(7);
constexpr int kWaitAllBut14Vmem = vmcnt_wait(14);

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

// Transpose-and-digitise: a workgroup of 16 S threads takes S consecutive
// slots of one (limb, entity) pair, where the entity is a query row (source:
// the query NTT form grouped by 32 slots, [L][R][N/32][d][32] uint64, so the
// workgroup's d x S words are d runs of S in one contiguous block) or a
// database chunk (source: the database residues [L][C][d][N] as 27-bit
// halves), stages the words in LDS, and writes each slot's 7 digit rows of
// Dp bytes (16 bytes per store, zero digits past coordinate d; two threads
// share a slot's 16-coordinate group, one for digits 0-3, one for 4-6).  The
// query side is read and written with nontemporal hints: it is touched once.
// LDS word (i, pp) sits at i (S + 1) + pp + i / 16: the extra word per 16
// coordinates puts the 16-coordinate groups that the lanes of one read
// instruction take on different banks (without it, eight of them share one).
template <bool DB, int S>
__global__ void __launch_bounds__(16 * S)
k_to_digits(const void* __restrict__ src, int8_t* __restrict__ dst, int n_ent, int d, int Dp,
            int L, int logN, int C, int Sk) {
  extern __shared__ uint64_t lw[];  // Dp (S + 1) + Dp / 16 words
  constexpr int P1 = S + 1, NT = 16 * S;
  auto at = [&](int i, int pp) { return i * P1 + pp + (i >> 4); };
  const int N = 1 << logN;
  const int groups = N / S;
  int b = blockIdx.x;
  const int pg = b % groups;
  b /= groups;
  const int ent = b % n_ent, l = b / n_ent;
  const int p0 = pg * S;
  const int tid = threadIdx.x;
  if constexpr (DB) {
    for (int idx = tid; idx < Dp * S; idx += NT) {
      const int i = idx / S, pp = idx % S;
      uint64_t x = 0;
      if (i < d) {
        const uint2 h = reinterpret_cast<const uint2*>(
            src)[(((size_t)l * C + ent) * d + i) * N + p0 + pp];
        x = (uint64_t)h.x + ((uint64_t)h.y << 27);
      }
      lw[at(i, pp)] = digit_word(x);
    }
  } else {
    // two consecutive slots of a coordinate per 16-byte load
    typedef uint64_t u64x2v __attribute__((ext_vector_type(2)));
    for (int idx = tid; idx < Dp * S / 2; idx += NT) {
      const int i = idx / (S / 2), pp = 2 * (idx % (S / 2));
      u64x2v x = {0, 0};
      if (i < d) {
        const int pq = p0 + pp;
        x = __builtin_nontemporal_load(reinterpret_cast<const u64x2v*>(
            reinterpret_cast<const uint64_t*>(src) +
            ((((size_t)l * n_ent + ent) * (N / kDigitGroup) + pq / kDigitGroup) * d + i) *
                kDigitGroup +
            pq % kDigitGroup));
      }
      lw[at(i, pp)] = digit_word(x.x);
      lw[at(i, pp) + 1] = digit_word(x.y);
    }
  }
  __syncthreads();
  const int cg_n = Dp / 16;
  typedef unsigned v4u __attribute__((ext_vector_type(4)));
  for (int u = tid; u < 2 * S * cg_n; u += NT) {
    const int hf = u & 1, cg = (u >> 1) % cg_n, pp = (u >> 1) / cg_n;
    const int p = p0 + pp;
    uint64_t y[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = lw[at(16 * cg + j, pp)];
    int8_t* row = DB ? dst + (((size_t)l * N + p) * C + ent) * Sk
                     : dst + (((size_t)l * N + p) * n_ent + ent) * (size_t)(7 * Dp);
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      const int a = hf ? 4 + aa : aa;
      if (a > 6) break;
      v4u v;
      v.x = gather_byte(y[0], y[1], y[2], y[3], a);
      v.y = gather_byte(y[4], y[5], y[6], y[7], a);
      v.z = gather_byte(y[8], y[9], y[10], y[11], a);
      v.w = gather_byte(y[12], y[13], y[14], y[15], a);
      __builtin_nontemporal_store(v, reinterpret_cast<v4u*>(row + a * Dp + 16 * cg));
    }
    if (DB && cg == 0 && hf == 0) *reinterpret_cast<uint4*>(row + 7 * Dp) = make_uint4(0, 0, 0, 0);
  }
}

__device__ __forceinline__ int32_t opaque_i32(int32_t x) {
  asm("" : "+v"(x));
  return x;
}

// A value below 2^58 congruent to V = sum_s S_s 256^s (Dp <= 256, so
// |S_s| < 2^29); k_sums_to_ct reduces it to [0, q):
//   g0 = S0 + S1 2^8 + S2 2^16 + S3 2^24          |g0| < 2^53
//   g1 = S4 + ... + S7 2^24  (weight 2^32)        |g1| < 2^53
//   h  = S8 + ... + S11 2^24 + S12 2^32  (weight 2^64),  |h| < 2^57
// and V = g0 + g1 2^32 + h 2^64.
__device__ __forceinline__ uint64_t fold_digit_sums(const int32_t (&S)[13],
                                                    const DigitConst& D) {
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
  return x0 + shoup_approx(x1, D.w32, D.w32p, D.nq) +
         shoup_approx(x2, D.w64, D.w64p, D.nq);  // < 2^55 + 8q < 2^58
}

// The same value for q = 2^54 - delta, 0 < delta < 2^22, without Shoup
// products (Dp <= 128, so |S_s| < 7 2^21 and |S_12| <= 2^19, as x_6, y_6 lie in
// [0, 64]).  With 2^54 = delta (mod q):
//   g0 = 2q + S0 + S1 2^8 + S2 2^16 + S3 2^24     |g0 - 2q| < 2^48
//   g1 = S4 + ... + S7 2^24,  h = S8 + ... + S11 2^24 + S12 2^32,  |h| < 2^52
// and V = g0 - 2q + 2^32 (g1 + 2^32 h).  Splitting h = 2^22 hh + hl
// (0 <= hl < 2^22):  2^32 h = 2^32 hl + 2^54 hh = 2^32 hl + delta hh, so
// V = g0 + 2^32 z (mod q) with z = g1 + 2^32 hl + delta hh in (-2^52, 2^54.2).
// Splitting z = 2^24 zh + zl (0 <= zl < 2^24, |zh| < 2^31):  2^32 z = 2^32 zl
// + 2^56 zh = 2^32 zl + 4 delta zh, and the result g0 + 2^32 zl + 4 delta zh
// lies in [0, 2^57).  Every product is one signed 32 x 32 -> 64-bit
// multiply-add.
__device__ __forceinline__ uint64_t fold_digit_sums_pm(const int32_t (&S)[13],
                                                       const DigitConst& D, int32_t k1,
                                                       int32_t k8, int32_t k16, int32_t k24) {
  auto group = [&](int s, int64_t base) {
    int64_t g = base + (int64_t)S[s] * k1;
    g += (int64_t)S[s + 1] * k8;
    g += (int64_t)S[s + 2] * k16;
    g += (int64_t)S[s + 3] * k24;
    return g;
  };
  const int64_t h = group(8, 0) + (int64_t)((uint64_t)(uint32_t)S[12] << 32);
  const int32_t hh = (int32_t)(uint32_t)((uint64_t)h >> 22);
  const uint32_t hl = (uint32_t)h & 0x3fffffu;
  const int64_t z = group(4, 0) + (int64_t)D.delta * hh + (int64_t)((uint64_t)hl << 32);
  const int32_t zh = (int32_t)(uint32_t)((uint64_t)z >> 24);
  const uint32_t zl = (uint32_t)z & 0xffffffu;
  const int64_t r = group(0, (int64_t)D.twoq) + (int64_t)(4 * D.delta) * zh +
                    (int64_t)((uint64_t)zl << 32);
  return (uint64_t)r;
}

// One MFMA step of the contraction: 64 coordinates (16 bytes per lane,
// v_mfma_i32_16x16x64_i8) or 32 (8 bytes per lane, v_mfma_i32_16x16x32_i8,
// lane l supplying row or column l % 16 and contraction bytes 8 (l / 16) ..
// + 7; the output layout is that of the 64-wide form).
template <bool W32>
struct StepFrag {
  typedef v4i T;
};
template <>
struct StepFrag<true> {
  typedef int64_t T;
};
template <bool W32>
__device__ __forceinline__ v4i mfma_digits(typename StepFrag<W32>::T a,
                                           typename StepFrag<W32>::T b, v4i c) {
  if constexpr (W32)
    return __builtin_amdgcn_mfma_i32_16x16x32_i8(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// One workgroup: 64 rows x 64 chunks of kMfmaSlots consecutive slots of one
// limb.  Wave w owns rows 16w .. 16w + 15 of the tile; its query fragments
// come straight from global memory into registers and serve the four
// 16-chunk column tiles of a slot.  The database digits are staged in LDS by
// DMA (global_load_lds) one column tile (stage) at a time, double-buffered
// in 2 x 16 KB, so that three workgroups fit on a CU (three waves per SIMD,
// at most 168 registers each; two workgroups of 32-chunk stages at 256
// registers ran 4-5% slower).  The DMA of the next stage is issued at the
// start of a stage, so it lands behind that stage's MFMAs (49 per
// 64-coordinate step), fold and stores.  Every memory operation of the loop is
// unconditional (the digit region has slack past its end, the sums buffer is
// padded to whole tiles): a stage's DMA may run up to 65 chunks past the last
// one (16 KB of reads from at most 47 chunks past it).  The query fragments
// of the next slot are loaded during the last stage of a slot, behind its
// MFMAs.  Before each barrier that publishes a buffer, a counted wait retires
// this wave's DMA into it (and nothing newer); the stores go out after the
// barrier.  The database fragments are plain LDS loads, which the compiler
// issues ahead of their MFMAs; empty asm statements with a memory clobber
// around each barrier keep them behind it.  Workgroups are numbered so that
// the tiles of one slot range run back to back on one XCD, which shares the
// operands in its L2.
template <int DP, bool PM>
__global__ void __launch_bounds__(256, 3)
k_mac_mfma(const int8_t* __restrict__ qd, const int8_t* __restrict__ dbd, int R, int C, int L,
             int logN, int n_items, DigitSet ds, uint64_t* __restrict__ sums) {
  constexpr int Dp = DP, Sk = 7 * Dp + 16, Dq = (Dp + 63) / 64 * 64;
  constexpr int NS = (Dp + 63) / 64;
  constexpr bool W0 = Dp < 64, W1 = Dp % 64 != 0;
  typedef typename StepFrag<W0>::T F0;
  typedef typename StepFrag<W1>::T F1;
  constexpr int H = 16;                 // chunks per stage
  constexpr int BU = H * Sk / 16;       // 16-byte units of one stage
  constexpr int BR = (BU + 255) / 256;  // DMA rounds of the 256 threads
  static_assert(BR * 256 * 16 + (kMfmaChunks - H) * Sk <= (int)kMfmaDbSlack,
                "a stage's DMA stays inside the digit region's slack");
  static_assert(!PM || Dp <= 128, "the bounds of the short fold hold for Dp <= 128");
  __shared__ uint4 sb0[BR * 256], sb1[BR * 256];
  const int N = 1 << logN;
  const int per_xcd = (n_items + 7) >> 3;
  const int lin = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lin >= n_items) return;
  const int nrt = (R + kMfmaRows - 1) / kMfmaRows, nct = (C + kMfmaChunks - 1) / kMfmaChunks;
  const int Rp = nrt * kMfmaRows, Cp = nct * kMfmaChunks;
  const int tile = lin % (nrt * nct), sg = lin / (nrt * nct);
  const int rt = tile % nrt, ctile = tile / nrt;
  const int l = sg % L, p0 = (sg / L) * kMfmaSlots;
  const int k0 = ctile * kMfmaChunks;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int m16 = lane & 15, g = lane >> 4;
  const int wrow0 = rt * kMfmaRows + 16 * w;
  const int arow = wrow0 + m16 < R ? wrow0 + m16 : R - 1;
  const DigitConst& D = ds.c[l];
  // opaque 1, 2^8, 2^16, 2^24: the fold's terms become 64-bit multiply-adds
  const int32_t k1 = opaque_i32(1), k8 = opaque_i32(1 << 8), k16 = opaque_i32(1 << 16),
                k24 = opaque_i32(1 << 24);
  auto stage = [&](int p, int cq, uint4* buf) {
    const uint4* src = reinterpret_cast<const uint4*>(
        dbd + (((size_t)l * N + p) * C + k0 + cq * H) * Sk);
#pragma unroll
    for (int m = 0; m < BR; ++m)
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + tid + 256 * m),
          (__attribute__((address_space(3))) void*)(buf + 256 * m + 64 * w), 16, 0, 0);
  };
  auto load_a = [&](int p, int ks, auto (&af)[7]) {
    typedef typename std::remove_reference<decltype(af[0])>::type F;
    const int8_t* ab = qd + (((size_t)l * N + p) * R + arow) * (size_t)(7 * Dq) +
                       (int)sizeof(F) * g + 64 * ks;
#pragma unroll
    for (int a = 0; a < 7; ++a) af[a] = *reinterpret_cast<const F*>(ab + a * Dq);
  };
  // 49 MFMAs of one step against the stage's column tile; the fragments are
  // plain LDS loads, which the compiler issues ahead of their MFMAs (the asm
  // clobbers at the barriers keep them after the barrier that publishes the
  // buffer)
  auto mfma_step = [&](const auto (&af)[7], int ks, const uint4* buf, v4i (&acc)[13]) {
    typedef typename std::remove_const<
        typename std::remove_reference<decltype(af[0])>::type>::type F;
    constexpr bool W = sizeof(F) == 8;
    const char* fb = reinterpret_cast<const char*>(buf) + m16 * Sk + (int)sizeof(F) * g + 64 * ks;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
      const F bf = *reinterpret_cast<const F*>(fb + b * Dp);
#pragma unroll
      for (int a = 0; a < 7; ++a)
        acc[a + b] = mfma_digits<W>(
            af[a], bf, (ks == 0 && (b == 0 || a == 6)) ? v4i{0, 0, 0, 0} : acc[a + b]);
    }
  };
  // one stage: quarter cq of slot p from buf, the next stage's DMA into nxt
  auto run_stage = [&](int p, int cq, const uint4* buf, uint4* nxt, int pn, F0 (&a0)[7],
                       F1 (&a1)[7]) {
    if (cq == 0) {
      // the slot's step-0 fragments: older than the step-1 loads (NS == 2)
      // and the previous stage's 4 stores
      __builtin_amdgcn_s_waitcnt(vmcnt_wait(NS == 2 ? 11 : 4));
      __builtin_amdgcn_sched_barrier(0);
    }
    if (cq < 3)
      stage(p, cq + 1, nxt);
    else
      stage(pn, 0, nxt);
    __builtin_amdgcn_sched_barrier(0);
    v4i acc[13];
    mfma_step(a0, 0, buf, acc);
    if constexpr (NS == 2) {
      if (cq == 0) {
        // the step-1 fragments: older than the stores and this stage's DMA
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(vmcnt_wait(4 + BR));
      }
      if (cq == 3) {
        __builtin_amdgcn_sched_barrier(0);
        load_a(pn, 0, a0);  // the next slot's step-0 fragments, behind step 1
      }
      __builtin_amdgcn_sched_barrier(0);
      mfma_step(a1, 1, buf, acc);
      if (cq == 3) {
        __builtin_amdgcn_sched_barrier(0);
        load_a(pn, 1, a1);
      }
    } else if (cq == 3) {
      __builtin_amdgcn_sched_barrier(0);
      load_a(pn, 0, a0);
    }
    __builtin_amdgcn_sched_barrier(0);
    uint64_t v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int32_t S[13];
#pragma unroll
      for (int s2 = 0; s2 < 13; ++s2) S[s2] = acc[s2][e];
      v[e] = PM ? fold_digit_sums_pm(S, D, k1, k8, k16, k24) : fold_digit_sums(S, D);
    }
    __builtin_amdgcn_sched_barrier(0);
    // the DMA into nxt: older than the fragment loads of a last stage
    if (cq == 3)
      __builtin_amdgcn_s_waitcnt(NS == 2 ? kWaitAllBut14Vmem : kWaitAllBut7Vmem);
    else
      __builtin_amdgcn_s_waitcnt(kWaitAllVmem);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    uint64_t* dst = sums + (((size_t)l * N + p) * Rp + wrow0 + 4 * g) * Cp + k0 + cq * H + m16;
#pragma unroll
    for (int e = 0; e < 4; ++e) __builtin_nontemporal_store(v[e], dst + (size_t)e * Cp);
  };

  F0 a0[7];
  F1 a1[7];
  stage(p0, 0, sb0);
  load_a(p0, 0, a0);
  if (NS == 2) load_a(p0, 1, a1);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int jj = 0; jj < kMfmaSlots; ++jj) {
    const int p = p0 + jj;
    const int pn = jj + 1 < kMfmaSlots ? p + 1 : p;  // the last slot restages itself
    run_stage(p, 0, sb0, sb1, pn, a0, a1);
    run_stage(p, 1, sb1, sb0, pn, a0, a1);
    run_stage(p, 2, sb0, sb1, pn, a0, a1);
    run_stage(p, 3, sb1, sb0, pn, a0, a1);
  }
}

// Slot-major sums [L][N][Rp][Cp] (values below 2^58) -> ciphertexts
// [Q C][2][L][N] reduced to [0, q) (output m = q C + k, component c = row & 1):
// 64 slots x 32 chunks of one row per workgroup.  The same launch draws the
// server masks of all Q C outputs (share != NULL): the ALU work of ChaCha20
// runs while this memory-bound transpose waits for its loads.  Mask blocks
// (four slots each, N / 4 per output) go in jobs of 64 consecutive blocks to
// whole waves: job j to wave j / gridDim.x of workgroup j mod gridDim.x (at
// most 4 jobs per workgroup, since there are at most C / (8 L ceil(C / 32))
// per workgroup).
__global__ void __launch_bounds__(256)
k_sums_to_ct(const uint64_t* __restrict__ sums, uint64_t* __restrict__ ct, int R, int C, int L,
             int logN, PrimeSet ps, MaskKey K, const uint64_t* __restrict__ qids, uint32_t t,
             uint64_t tone, uint32_t* __restrict__ share) {
  __shared__ uint64_t tb[32][65];
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
  const int Rp = (R + kMfmaRows - 1) / kMfmaRows * kMfmaRows;
  const int Cp = (C + kMfmaChunks - 1) / kMfmaChunks * kMfmaChunks;
  // two consecutive chunks of a slot per 16-byte load (Cp is a multiple of 64)
  typedef uint64_t u64x2v __attribute__((ext_vector_type(2)));
  u64x2v x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i, kk = 2 * (idx % 16), pp = idx / 16;
    x[i] = __builtin_nontemporal_load(reinterpret_cast<const u64x2v*>(
        sums + (((size_t)l * N + p0 + pp) * Rp + row) * Cp + k0 + kk));
  }
  if (share) {
    const int nb = N >> 2;
    const long n_blocks = (long)(R >> 1) * C * nb;
    const long blk = ((long)blockIdx.x + (long)(tid >> 6) * gridDim.x) * 64 + (tid & 63);
    if (blk < n_blocks) {
      const int m = (int)(blk / nb), bb = (int)(blk % nb);
      mask_block(K, qids[m / C], m % C, bb, t, tone, share + (size_t)m * N);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i, kk = 2 * (idx % 16), pp = idx / 16;
    tb[kk][pp] = x[i].x;
    tb[kk + 1][pp] = x[i].y;
  }
  __syncthreads();
  const int q = row >> 1, c = row & 1;
  const Prime& P = ps.p[l];
  const uint64_t nq = 0 - P.q;
  // x < 2^58 -> [0, q): for q = 2^54 - delta with delta < 2^22 by 2^54 =
  // delta (mod q), else by a Shoup product by 1 (to [0, 4q)) and two
  // conditional subtractions
  const uint32_t pd = pm_delta(P.q);
  auto reduce = [&](uint64_t x) -> uint64_t {
    if (pd) return reduce_pm60(x, pd, P.q);
    return csub(csub(shoup_approx(x, 1, P.one, nq), 2 * P.q), P.q);
  };
  // two consecutive slots per 16-byte store
  for (int idx = tid; idx < 32 * 32; idx += 256) {
    const int pp = 2 * (idx % 32), kk = idx / 32;
    if (k0 + kk < C) {
      const u64x2v v = {reduce(tb[kk][pp]), reduce(tb[kk][pp + 1])};
      __builtin_nontemporal_store(
          v, reinterpret_cast<u64x2v*>(
                 ct + ((((size_t)q * C + k0 + kk) * 2 + c) * L + l) * N + p0 + pp));
    }
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

int mfma_padded_d(int d) { return (d + 31) / 32 * 32; }
int mfma_query_d(int d) { return (d + 63) / 64 * 64; }
size_t mfma_sums_bytes(int Q, int C, int L, int logN) {
  const size_t Rp = (2 * (size_t)Q + kMfmaRows - 1) / kMfmaRows * kMfmaRows;
  const size_t Cp = ((size_t)C + kMfmaChunks - 1) / kMfmaChunks * kMfmaChunks;
  return (size_t)L * ((size_t)1 << logN) * Rp * Cp * sizeof(uint64_t);
}
int mfma_db_stride(int d) { return 7 * mfma_padded_d(d) + 16; }
size_t mfma_db_bytes(int C, int d, int L, int logN) {
  return (size_t)L * ((size_t)1 << logN) * C * mfma_db_stride(d) + kMfmaDbSlack;
}

bool mfma_supported(int logN, int d) {
  return logN >= 6 && d >= 1 && d <= kMfmaMaxD;
}

hipError_t launch_query_digits(const uint64_t* qntt, int8_t* qd, int Q, int d, int L, int logN,
                               hipStream_t st) {
  const int Dp = mfma_query_d(d), N = 1 << logN;
  constexpr int S = kQueryDigitSlots;
  const long nb = (long)L * 2 * Q * (N / S);
  if (nb <= 0) return hipSuccess;
  const size_t lds = ((size_t)Dp * (S + 1) + Dp / 16) * sizeof(uint64_t);
  hipLaunchKernelGGL((k_to_digits<false, S>), dim3((unsigned)nb), dim3(16 * S), lds, st,
                     (const void*)qntt, qd, 2 * Q, d, Dp, L, logN, 0, 0);
  return hipGetLastError();
}

hipError_t launch_db_digits(const uint2* dbres, int8_t* dbd, int C, int d, int L, int logN,
                            hipStream_t st) {
  const int Dp = mfma_padded_d(d), N = 1 << logN;
  const long nb = (long)L * C * (N / 32);
  if (nb <= 0) return hipSuccess;
  const size_t lds = ((size_t)Dp * (32 + 1) + Dp / 16) * sizeof(uint64_t);
  hipLaunchKernelGGL((k_to_digits<true, 32>), dim3((unsigned)nb), dim3(512), lds, st,
                     (const void*)dbres, dbd, C, d, Dp, L, logN, C, mfma_db_stride(d));
  return hipGetLastError();
}

template <int DP>
static void launch_mac_mfma_t(const int8_t* qd, const int8_t* dbd, int R, int C, int L, int logN,
                              const DigitSet& ds, uint64_t* sums, hipStream_t st) {
  const int N = 1 << logN;
  const long n_items = (long)L * (N / kMfmaSlots) * ((R + kMfmaRows - 1) / kMfmaRows) *
                       ((C + kMfmaChunks - 1) / kMfmaChunks);
  const long per_xcd = (n_items + 7) >> 3;
  // the short fold when every prime is 2^54 - delta with a small delta
  bool pm = true;
  for (int l = 0; l < L; ++l) pm = pm && ds.c[l].delta != 0;
  if (pm)
    hipLaunchKernelGGL((k_mac_mfma<DP, true>), dim3((unsigned)(per_xcd * 8)), dim3(256), 0, st,
                       qd, dbd, R, C, L, logN, (int)n_items, ds, sums);
  else
    hipLaunchKernelGGL((k_mac_mfma<DP, false>), dim3((unsigned)(per_xcd * 8)), dim3(256), 0, st,
                       qd, dbd, R, C, L, logN, (int)n_items, ds, sums);
}

hipError_t launch_mac_mfma(const int8_t* qd, const int8_t* dbd, int Q, int d, int C, int L,
                           int logN, const DigitSet& ds, uint64_t* sums, hipStream_t st) {
  if (!mfma_supported(logN, d)) return hipErrorInvalidValue;
  if (Q <= 0 || C <= 0) return hipSuccess;
  const int R = 2 * Q;
  switch (mfma_padded_d(d)) {
    case 32: launch_mac_mfma_t<32>(qd, dbd, R, C, L, logN, ds, sums, st); break;
    case 64: launch_mac_mfma_t<64>(qd, dbd, R, C, L, logN, ds, sums, st); break;
    case 96: launch_mac_mfma_t<96>(qd, dbd, R, C, L, logN, ds, sums, st); break;
    case 128: launch_mac_mfma_t<128>(qd, dbd, R, C, L, logN, ds, sums, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sums_to_ct(const uint64_t* sums, uint64_t* ct_out, int Q, int C, int L,
                             int logN, const PrimeSet& ps, hipStream_t st, const MaskKey& K,
                             const uint64_t* qids, uint32_t t, uint64_t tone, uint32_t* share) {
  if (logN < 6) return hipErrorInvalidValue;
  if (Q <= 0 || C <= 0) return hipSuccess;
  const int R = 2 * Q, N = 1 << logN;
  const long nb = (long)L * (N / 64) * R * ((C + 31) / 32);
  // the mask jobs must fit in the workgroups' four waves
  if (share && ((long)Q * C * (N / 4) + 63) / 64 > 4 * nb) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sums_to_ct, dim3((unsigned)nb), dim3(256), 0, st, sums, ct_out, R, C, L,
                     logN, ps, K, qids, t, tone, share);
  return hipGetLastError();
}

}  // namespace sanns
