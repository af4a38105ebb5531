// Device modular arithmetic for residues below 2^54, built from the 32-bit
// multiplier (v_mul_hi_u32, v_mul_lo_u32, v_mad_u64_u32 all issue at full
// rate on gfx950, so every wide product below is spelled out in 32-bit
// pieces).
//
// Shoup multiplication by a fixed operand w < q with companion
// w' = floor(w * 2^64 / q):  for any x < 2^64,
//     Qhat = floor(x w' / 2^64)  and  r = x w - Qhat q  (mod 2^64)
// satisfy 0 <= r < 2q, because x w / q - Qhat < x / 2^64 + 1 < 2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sanns {

typedef HIP_vector_type<unsigned long long, 2> u64x2;  // (w, Shoup companion)

__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }

__device__ __forceinline__ uint64_t mul32x32(uint32_t a, uint32_t b) {
  return (uint64_t)a * b;
}

// Exact floor(x * y / 2^64).
__device__ __forceinline__ uint64_t mulhi64(uint64_t x, uint64_t y) {
  uint32_t x0 = lo32(x), x1 = hi32(x), y0 = lo32(y), y1 = hi32(y);
  uint64_t t = mul32x32(x0, y1) + __umulhi(x0, y0);  // < 2^64
  uint64_t u = mul32x32(x1, y0) + lo32(t);           // < 2^64
  return mul32x32(x1, y1) + hi32(t) + hi32(u);
}

// x * y mod 2^64.
__device__ __forceinline__ uint64_t mullo64(uint64_t x, uint64_t y) {
  uint32_t x0 = lo32(x), x1 = hi32(x), y0 = lo32(y), y1 = hi32(y);
  uint64_t p = mul32x32(x0, y0);
  uint32_t cross = x0 * y1 + x1 * y0;
  return p + ((uint64_t)cross << 32);
}

// Shoup product in [0, 2q) for any x < 2^64.
__device__ __forceinline__ uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t wp,
                                               uint64_t q) {
  uint64_t Q = mulhi64(x, wp);
  return mullo64(x, w) - mullo64(Q, q);
}

__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t q) {
  // x - q with the borrow chain's final borrow selecting the result
  unsigned b0, b1;
  const uint32_t lo = __builtin_subc(lo32(x), lo32(q), 0u, &b0);
  const uint32_t hi = __builtin_subc(hi32(x), hi32(q), b0, &b1);
  return b1 ? x : (((uint64_t)hi << 32) | lo);
}

// The 32-bit halves of a value, hidden from the optimiser so that products
// spelled out below in 32-bit pieces stay as written instead of being folded
// back into a generic 64-bit multiply (an empty asm statement, no code).
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm("" : "+v"(x));
  return x;
}

// Shoup product with the quotient estimated from three of the four 32-bit
// partial products of x w' (x0 p0 and the low halves of x1 p0 and x0 p1 are
// dropped, which lowers the estimate by at most 2), and x w - Qhat q formed
// as x w + Qhat nq with nq = 2^64 - q.  Result in [0, 4q) for x < 2^62.
__device__ __forceinline__ uint64_t shoup_approx(uint64_t x, uint64_t w, uint64_t wp,
                                                 uint64_t nq) {
  const uint32_t x0 = opaque(lo32(x)), x1 = opaque(hi32(x));
  const uint32_t p0 = lo32(wp), p1 = hi32(wp);
  const uint64_t qh = mul32x32(x1, p1) + __umulhi(x1, p0) + __umulhi(x0, p1);
  const uint32_t q0 = opaque(lo32(qh)), q1 = opaque(hi32(qh));
  const uint64_t lo = mul32x32(x0, lo32(w)) + mul32x32(q0, lo32(nq));
  const uint32_t hi = hi32(lo) + x0 * hi32(w) + x1 * lo32(w) + q0 * hi32(nq) + q1 * lo32(nq);
  return ((uint64_t)hi << 32) | lo32(lo);
}

// Shoup product reduced to [0, q).
__device__ __forceinline__ uint64_t shoup(uint64_t x, uint64_t w, uint64_t wp,
                                          uint64_t q) {
  return csub(shoup_lazy(x, w, wp, q), q);
}

// x mod q for any x < 2^64, with one = floor(2^64 / q) (Shoup with w = 1).
__device__ __forceinline__ uint64_t reduce64(uint64_t x, uint64_t one, uint64_t q) {
  uint64_t r = x - mullo64(mulhi64(x, one), q);
  return csub(r, q);
}

// delta when q = 2^54 - delta with 0 < delta < 2^22, else 0.
__host__ __device__ inline uint32_t pm_delta(uint64_t q) {
  const uint64_t two54 = 1ull << 54;
  return (q < two54 && two54 - q < (1ull << 22)) ? (uint32_t)(two54 - q) : 0u;
}

// x mod q for x < 2^60 and q = 2^54 - delta, delta = pm_delta(q) != 0: with
// 2^54 = delta (mod q), x mod 2^54 + (x >> 54) delta < 2^54 + 2^28 < 2q, then
// one conditional subtraction.
__device__ __forceinline__ uint64_t reduce_pm60(uint64_t x, uint32_t delta, uint64_t q) {
  const uint64_t r = (uint64_t)(uint32_t)(x >> 54) * delta + (x & ((1ull << 54) - 1));
  return csub(r, q);
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
  return csub(a + b, q);
}
__device__ __forceinline__ uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
  return a >= b ? a - b : a + q - b;
}

// Constants of one RNS prime, passed to kernels by value.
struct Prime {
  uint64_t q;
  uint64_t one;      // floor(2^64 / q)
  uint64_t c54;      // 2^54 mod q
  uint64_t c54p;     // Shoup companion of c54
  uint64_t delta;    // floor(Q / t) mod q   (Q the whole modulus)
  uint64_t deltap;   // Shoup companion of delta
  uint64_t ninv;     // N^-1 mod q
  uint64_t ninvp;
};

// Multiply-accumulate of 54-bit residues in 27-bit halves (Karatsuba):
// a = a1 2^27 + a0, b = b1 2^27 + b0,
//   a b = a1 b1 2^54 + ((a0 + a1)(b0 + b1) - a0 b0 - a1 b1) 2^27 + a0 b0.
// Each product is below 2^56, so up to 255 terms fit the 64-bit sums.
struct Acc3 {
  uint64_t lo, mid, hi;
};

__device__ __forceinline__ void acc3_zero(Acc3 &a) { a.lo = a.mid = a.hi = 0; }

// Fold an accumulator into a residue in [0, q):
//   V = hi 2^54 + (mid - lo - hi) 2^27 + lo = H 2^54 + W  with
//   H = hi + (m >> 27), W = (m mod 2^27) 2^27 + lo, both below 2^64.
__device__ __forceinline__ uint64_t acc3_reduce(const Acc3 &a, const Prime &P) {
  uint64_t m = a.mid - a.lo - a.hi;
  uint64_t H = a.hi + (m >> 27);
  uint64_t W = ((m & ((1ull << 27) - 1)) << 27) + a.lo;
  uint64_t r = shoup_lazy(H, P.c54, P.c54p, P.q) + shoup_lazy(W, 1, P.one, P.q);
  r = csub(r, 2 * P.q);
  return csub(r, P.q);
}

__device__ __forceinline__ void split27(uint64_t x, uint32_t &x0, uint32_t &x1) {
  x0 = lo32(x) & ((1u << 27) - 1);
  x1 = (uint32_t)(x >> 27);
}

}  // namespace sanns
