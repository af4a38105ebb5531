// Host-side launchers of the kernels in kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"

namespace sanns {

// (QT, CT) register tiles of the multiply-accumulate kernel that are built.
#define SANNS_MAC_SHAPES(X) \
  X(1, 1) X(1, 2) X(1, 4) X(1, 8) X(2, 2) X(2, 4) X(4, 2) X(2, 3) X(3, 2)

// split: output form of the NTT residues (0 plain, 1 27-bit halves for the
// 64-bit multiply-accumulate kernels, 2 grouped by 32 slots for the digit
// transpose, which needs d and R = 2Q with n_polys = R d L).
hipError_t launch_ntt_fwd(const uint64_t* in, uint64_t* out, int n_polys, int logN, int L,
                          const PrimeSet& ps, const TwSet& tws, uint32_t* err, int split,
                          hipStream_t st, int d = 0, int R = 0);
hipError_t launch_ntt_inv(uint64_t* io, int n_polys, int logN, int L, const PrimeSet& ps,
                          const TwSet& tws, hipStream_t st);
hipError_t launch_masks(const MaskKey& K, const uint64_t* qids, const uint32_t* work, int C,
                        int M, int logN, uint32_t t, uint64_t tone, uint32_t* share,
                        hipStream_t st);
hipError_t launch_intt_mask(uint64_t* ct, const uint32_t* share, const uint32_t* norms,
                            const uint32_t* work, int C, int M, int logN, int L, uint32_t t,
                            const PrimeSet& ps, const TwSet& tws, hipStream_t st);
// tiles == NULL: every query against every chunk (Q x C outputs, m = q C + k).
hipError_t launch_mac(int QT, int CT, const uint2* qntt, const uint2* db, const void* tiles,
                      int n_tiles, int Q, int d, int L, int logN, int C, const PrimeSet& ps,
                      uint64_t* out, hipStream_t st);
size_t mac_tile_bytes(int QT, int CT);  // 0 for a shape that is not built

// LDS-staged variants of the all-pairs multiply-accumulate:
// X(id, QT, CT, QG, CG, S, DI, UNR), block = S slots x QG x CG threads
// covering QG QT queries x CG CT chunks, DI coordinates per staging step,
// UNR = unroll of the coordinate loop.
#define SANNS_MAC_LDS_VARIANTS(X)      \
  X(1, 2, 4, 4, 4, 32, 4, 2)           \
  X(2, 2, 4, 4, 4, 32, 4, 1)           \
  X(3, 2, 3, 4, 4, 32, 4, 2)           \
  X(4, 2, 3, 4, 4, 32, 4, 1)           \
  X(5, 2, 2, 4, 4, 32, 4, 2)           \
  X(6, 1, 4, 8, 4, 32, 4, 2)           \
  X(7, 2, 4, 4, 4, 32, 8, 1)           \
  X(8, 2, 3, 4, 4, 32, 8, 1)           \
  X(9, 2, 4, 2, 4, 32, 4, 1)           \
  X(10, 2, 4, 4, 2, 32, 4, 1)          \
  X(11, 2, 3, 2, 4, 32, 4, 1)
// Direct-to-LDS variants (same parameters), ids 21 and up.
#define SANNS_MAC_DL_VARIANTS(X)       \
  X(21, 2, 4, 4, 4, 32, 4, 1)          \
  X(22, 2, 4, 2, 4, 32, 4, 1)          \
  X(23, 1, 4, 8, 4, 32, 4, 2)          \
  X(24, 2, 4, 4, 4, 32, 8, 1)          \
  X(25, 2, 3, 4, 4, 32, 8, 1)          \
  X(26, 2, 4, 2, 4, 32, 8, 1)          \
  X(27, 2, 6, 2, 4, 32, 4, 1)
hipError_t launch_mac_lds(int variant, const uint2* qntt, const uint2* db, int Q, int d, int L,
                          int logN, int C, const PrimeSet& ps, uint64_t* out, hipStream_t st);
int mac_lds_min_n(int variant);  // slots per block (N must be a multiple); 0 if unknown
// Shapes of the persistent whole-batch kernel:
// X(id, LOGN, QT, CT, QG, CG, DI): one workgroup of N/16 threads per item; the
// multiply-accumulate tiles are direct-to-LDS tiles of QG QT queries x CG CT
// chunks over S = N / (16 QG CG) slots.  Work lists use 2 x 2 register tiles.
#define SANNS_PERSIST_SHAPES(X)          \
  X(41, 13, 2, 2, 4, 4, 4)               \
  X(42, 13, 1, 4, 4, 4, 4)               \
  X(43, 13, 2, 2, 2, 8, 4)               \
  X(44, 13, 1, 4, 8, 2, 4)               \
  X(51, 12, 2, 2, 2, 4, 4)               \
  X(52, 12, 1, 4, 2, 4, 4)               \
  X(61, 11, 2, 2, 1, 4, 4)               \
  X(71, 14, 2, 2, 4, 4, 2)
constexpr int kPersistTileQ = 2, kPersistTileC = 2;
constexpr int kPersistCtrlWords = 16;
int persistent_logn(int shape);           // 0 if the shape is not built
int persistent_default_shape(int logN);   // 0 if N is not supported
int persistent_max_d(int shape);          // largest d the shape accumulates in one pass
hipError_t launch_persistent(int shape, const PersistArgs& A, const PrimeSet& ps,
                             const TwSet& tws, hipStream_t st);

// Matrix-core schedule of the all-pairs multiply-accumulate (mfma.hip).
constexpr int kMfmaSchedule = 81;  // schedule id of sanns_set_schedule
constexpr int kMfmaMaxD = 128;     // largest d (two MFMA steps of 64 coordinates)
bool mfma_supported(int logN, int d);
int mfma_padded_d(int d);   // d rounded up to 32: database digit rows, contraction
int mfma_query_d(int d);    // d rounded up to 64: query digit rows
int mfma_db_stride(int d);  // bytes per (limb, slot, chunk) of the database digits
size_t mfma_db_bytes(int C, int d, int L, int logN);  // the digit region, with its slack
// Query NTT form grouped by 32 slots ([L][2Q][N/32][d][32] uint64, NTT output
// form 2) -> query digits [L][N][2Q][7][Dq], Dq = mfma_query_d(d).
hipError_t launch_query_digits(const uint64_t* qntt, int8_t* qd, int Q, int d, int L, int logN,
                               hipStream_t st);
// Database residues [L][C][d][N] (halves) -> database digits [L][N][C][Sk].
hipError_t launch_db_digits(const uint2* dbres, int8_t* dbd, int C, int d, int L, int logN,
                            hipStream_t st);
// All-pairs sums into the slot-major buffer `sums` ([L][N][Rp][Cp] uint64
// below 2^58, Rp = 2Q and Cp = C rounded up to 64; mfma_sums_bytes).
size_t mfma_sums_bytes(int Q, int C, int L, int logN);
hipError_t launch_mac_mfma(const int8_t* qd, const int8_t* dbd, int Q, int d, int C, int L,
                           int logN, const DigitSet& ds, uint64_t* sums, hipStream_t st);
// The sums reduced to [0, q) and transposed into ct_out [Q C][2][L][N] (NTT
// form); with share != NULL the same launch writes the server masks of the
// Q C outputs (output m = q C + k), as launch_masks does.
hipError_t launch_sums_to_ct(const uint64_t* sums, uint64_t* ct_out, int Q, int C, int L,
                             int logN, const PrimeSet& ps, hipStream_t st, const MaskKey& K,
                             const uint64_t* qids, uint32_t t, uint64_t tone, uint32_t* share);

hipError_t launch_gather(const void* pts, int is_signed, long n, int d,
                         const int64_t* slot_point, long base, long total, int logN,
                         int16_t* gt, uint32_t* norms, uint32_t* err, hipStream_t st);
// Slot map of gathered chunks from point ranges: -1 everywhere, then
// slot[off[r] + i] = start[r] + i, i < len[r].
hipError_t launch_slot_ranges(const int64_t* start, const int64_t* len, const int64_t* off,
                              int R, int64_t* slot, long total, hipStream_t st);
// Gathered chunks: kind 0 / 1 uint8 / int8 points, 2 shares in [0, t) with
// their norm shares; 32-bit plaintext coefficients.
hipError_t launch_gather32(const void* pts, int kind, long n, int d, const uint32_t* norm_shares,
                           uint32_t t, const int64_t* slot_point, long base, long total,
                           int logN, int32_t* gt, uint32_t* norms, uint32_t* err,
                           hipStream_t st);
hipError_t launch_encode_ntt32(const int32_t* gt, uint2* dbres, int k0, int nk, int C, int d,
                               int logN, int L, const PrimeSet& ps, const TwSet& tws,
                               hipStream_t st);
hipError_t launch_encode_ntt(const int16_t* gt, uint2* dbres, int k0, int nk, int C, int d,
                             int logN, int L, const PrimeSet& ps, const TwSet& tws,
                             hipStream_t st);
hipError_t launch_sk_ntt(const int8_t* sk, uint64_t* out, int logN, int L, const PrimeSet& ps,
                         const TwSet& tws, hipStream_t st);
// k-means of the balanced clustering (kmeans.hip): int8 points [n][d]
// (d <= 256), centres int32 [k][d] on a 2^-8 grid; workspace km_workspace().
size_t km_workspace(int k, int d);
hipError_t launch_km_init(const int8_t* X, long n, int d, const int64_t* idx, int k, int32_t* C,
                          uint32_t* bad, hipStream_t st);
hipError_t launch_km_assign(const int8_t* X, long n, int d, const int32_t* C, int k,
                            const int32_t* prev, int32_t* assign, uint32_t* changed, void* ws,
                            hipStream_t st);
hipError_t launch_km_update(const int8_t* X, long n, int d, const int32_t* assign, int k,
                            int32_t* C, int64_t* counts_out, void* ws, hipStream_t st);

// Client randomness from a seed: ternary secret [N]; uniform a [Qd][L][N]
// and errors e [Qd][N] of Qd = Q d encrypted coordinates.
hipError_t launch_keygen(uint64_t seed, int N, int8_t* sk, hipStream_t st);
hipError_t launch_sample_enc(uint64_t seed, uint32_t purpose_a, uint32_t purpose_e, int Qd,
                             int d, int L, int N, const PrimeSet& ps, uint64_t* a, int16_t* e,
                             hipStream_t st);
// Circuit privacy: u pk added to the NTT-form outputs (pk_ntt [Q][2][L][N] in
// NTT storage order), then the inverse transform with e1, flood and the mask
// plaintext on c0 and e2 on c1.
hipError_t launch_rerand(const MaskKey& K, const uint64_t* qids, const uint32_t* work, int C,
                         int M, int L, int logN, const uint64_t* pk_ntt, uint64_t* ct,
                         const PrimeSet& ps, const TwSet& tws, hipStream_t st);
// flood: workspace [M][L][N] uint64 for the flood residues, followed by
// [M][2][N] int8 for e1 and e2 (k_cp_noise).
hipError_t launch_intt_mask_cp(uint64_t* ct, const uint32_t* share, const uint32_t* norms,
                               const uint32_t* work, int C, int M, int logN, int L, uint32_t t,
                               const MaskKey& K, const uint64_t* qids, const CpConst& cp,
                               const DigitSet& ds, const PrimeSet& ps, const TwSet& tws,
                               uint64_t* flood, hipStream_t st);
hipError_t launch_encrypt(const uint64_t* a, const int16_t* e, const int32_t* msgs,
                          const uint64_t* sk_ntt, uint64_t* ct, int Qd, int L, int logN,
                          uint32_t t, const PrimeSet& ps, const TwSet& tws, hipStream_t st);
hipError_t launch_decrypt(const uint64_t* ct, int M, const uint64_t* sk_ntt,
                          const uint32_t* qnorm2, uint32_t* out, int L, int logN,
                          const PrimeSet& ps, const TwSet& tws, const DecodeConst& D,
                          hipStream_t st);
hipError_t launch_mult_plain(const uint2* cq, const uint2* db, int i, int k, int d, int C,
                             int L, int logN, const PrimeSet& ps, uint64_t* tmp,
                             hipStream_t st);
hipError_t launch_add(uint64_t* acc, const uint64_t* tmp, int L, int logN, const PrimeSet& ps,
                      hipStream_t st);
hipError_t launch_add_plain(uint64_t* ct, const uint32_t* share, const uint32_t* norms, int k,
                            int L, int logN, uint32_t t, const PrimeSet& ps, hipStream_t st);

}  // namespace sanns
