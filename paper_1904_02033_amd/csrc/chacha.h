// ChaCha20 block function (RFC 8439, Section 2.3) and the server's masks
// drawn from it (Section 4.2: uniform Z_t randomness that turns each
// distance into additive shares): shared by the kernels of both files.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "modarith.h"

namespace sanns {

__device__ __forceinline__ uint32_t rotl(uint32_t x, int n) {
  return __builtin_rotateleft32(x, n);
}

#define SANNS_QR(a, b, c, d)          \
  a += b; d ^= a; d = rotl(d, 16);    \
  c += d; b ^= c; b = rotl(b, 12);    \
  a += b; d ^= a; d = rotl(d, 8);     \
  c += d; b ^= c; b = rotl(b, 7);

__device__ __forceinline__ void chacha_block(const MaskKey& K, uint32_t ctr, uint32_t n0,
                                             uint32_t n1, uint32_t n2, uint32_t (&o)[16]) {
  uint32_t x0 = 0x61707865u, x1 = 0x3320646eu, x2 = 0x79622d32u, x3 = 0x6b206574u;
  uint32_t x4 = K.k[0], x5 = K.k[1], x6 = K.k[2], x7 = K.k[3];
  uint32_t x8 = K.k[4], x9 = K.k[5], x10 = K.k[6], x11 = K.k[7];
  uint32_t x12 = ctr, x13 = n0, x14 = n1, x15 = n2;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    SANNS_QR(x0, x4, x8, x12) SANNS_QR(x1, x5, x9, x13)
    SANNS_QR(x2, x6, x10, x14) SANNS_QR(x3, x7, x11, x15)
    SANNS_QR(x0, x5, x10, x15) SANNS_QR(x1, x6, x11, x12)
    SANNS_QR(x2, x7, x8, x13) SANNS_QR(x3, x4, x9, x14)
  }
  o[0] = x0 + 0x61707865u; o[1] = x1 + 0x3320646eu;
  o[2] = x2 + 0x79622d32u; o[3] = x3 + 0x6b206574u;
  o[4] = x4 + K.k[0]; o[5] = x5 + K.k[1]; o[6] = x6 + K.k[2]; o[7] = x7 + K.k[3];
  o[8] = x8 + K.k[4]; o[9] = x9 + K.k[5]; o[10] = x10 + K.k[6]; o[11] = x11 + K.k[7];
  o[12] = x12 + ctr; o[13] = x13 + n0; o[14] = x14 + n1; o[15] = x15 + n2;
}
#undef SANNS_QR

// (w3 2^96 + w2 2^64 + w1 2^32 + w0) mod t by Horner steps below 2^63.
__device__ __forceinline__ uint32_t mod_t_128(uint32_t w0, uint32_t w1, uint32_t w2,
                                              uint32_t w3, uint32_t t, uint64_t tone) {
  uint64_t r = reduce64(w3, tone, t);
  r = reduce64((r << 32) | w2, tone, t);
  r = reduce64((r << 32) | w1, tone, t);
  r = reduce64((r << 32) | w0, tone, t);
  return (uint32_t)r;
}


// Masks of slots 4b .. 4b+3 of output row m (query id, chunk k).
__device__ __forceinline__ void mask_block(const MaskKey& K, uint64_t id, int k, int b,
                                           uint32_t t, uint64_t tone, uint32_t* __restrict__ row) {
  uint32_t o[16];
  chacha_block(K, (uint32_t)b, (uint32_t)id, (uint32_t)(id >> 32), (uint32_t)k, o);
  uint4 r;
  r.x = mod_t_128(o[0], o[1], o[2], o[3], t, tone);
  r.y = mod_t_128(o[4], o[5], o[6], o[7], t, tone);
  r.z = mod_t_128(o[8], o[9], o[10], o[11], t, tone);
  r.w = mod_t_128(o[12], o[13], o[14], o[15], t, tone);
  reinterpret_cast<uint4*>(row)[b] = r;
}

}  // namespace sanns
