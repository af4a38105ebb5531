// k-means of the balanced clustering (Section 3.3; Lloyd's k-means, Section
// 2) on int8 points with centres on a grid of 2^-8, in exact integer
// arithmetic:
//   assignment  argmin_j ||2^8 x - C_j||^2 = argmin_j ( ||C_j||^2 - 2^9 <x, C_j> ),
//               ties to the lower index.  <x, C_j> is formed with 4-way int8
//               dot products on the two signed base-256 digits of C_j
//               (C = 256 hi + lo, lo in [-128, 127]); every partial sum
//               stays within int32 for d <= 256.
//   update      centre j = floor(2^8 S_j / n_j + 1/2) from exact 64-bit
//               sums (integer atomics, so the order of the additions does
//               not matter); an empty cluster keeps its centre.
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "launch.h"

namespace sanns {

constexpr int kKmTile = 32;     // centres per LDS tile
constexpr int kKmPoints = 2;    // points per thread

// Centre j as digit words: hi[w], then lo[w], w < DW (4 coordinates per
// word, zero past d), and ||C_j||^2.
__global__ void __launch_bounds__(256)
k_km_pack(const int32_t* __restrict__ C, int k, int d, int dw, int32_t* __restrict__ packed,
          int64_t* __restrict__ cnorm) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const int32_t* c = C + (size_t)j * d;
  int32_t* hi = packed + (size_t)j * 2 * dw;
  int32_t* lo = hi + dw;
  int64_t nrm = 0;
  for (int w = 0; w < dw; ++w) {
    uint32_t h = 0, l = 0;
    for (int b = 0; b < 4; ++b) {
      const int i = 4 * w + b;
      const int v = i < d ? c[i] : 0;
      const int lv = ((v + 128) & 255) - 128;
      const int hv = (v - lv) / 256;
      l |= (uint32_t)(uint8_t)(int8_t)lv << (8 * b);
      h |= (uint32_t)(uint8_t)(int8_t)hv << (8 * b);
      nrm += (int64_t)v * v;
    }
    hi[w] = (int32_t)h;
    lo[w] = (int32_t)l;
  }
  cnorm[j] = nrm;
}

// Thread per kKmPoints points (strided by the workgroup size); the centres
// pass through LDS kKmTile at a time (every lane reads the same words).
template <int DW>
__global__ void __launch_bounds__(256)
k_km_assign(const int8_t* __restrict__ X, long n, int d, const int32_t* __restrict__ packed,
            const int64_t* __restrict__ cnorm, int k, const int32_t* __restrict__ prev,
            int32_t* __restrict__ assign, uint32_t* __restrict__ changed) {
  __shared__ int32_t cw[kKmTile][2 * DW];
  __shared__ int64_t cn[kKmTile];
  const int tid = threadIdx.x;
  const long base = (long)blockIdx.x * 256 * kKmPoints;
  int32_t x[kKmPoints][DW];
  int64_t best[kKmPoints];
  int bi[kKmPoints];
#pragma unroll
  for (int p = 0; p < kKmPoints; ++p) {
    const long pt = base + tid + 256 * p;
    const int8_t* row = X + (pt < n ? pt : 0) * (long)d;
#pragma unroll
    for (int w = 0; w < DW; ++w) {
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = 4 * w + b;
        if (i < d) v |= (uint32_t)(uint8_t)row[i] << (8 * b);
      }
      x[p][w] = (int32_t)v;
    }
    best[p] = INT64_MAX;
    bi[p] = 0;
  }
  for (int c0 = 0; c0 < k; c0 += kKmTile) {
    const int nt = k - c0 < kKmTile ? k - c0 : kKmTile;
    __syncthreads();
    for (int u = tid; u < nt * 2 * DW; u += 256)
      cw[u / (2 * DW)][u % (2 * DW)] = packed[(size_t)(c0 + u / (2 * DW)) * 2 * DW + u % (2 * DW)];
    for (int u = tid; u < nt; u += 256) cn[u] = cnorm[c0 + u];
    __syncthreads();
    for (int c = 0; c < nt; ++c) {
#pragma unroll
      for (int p = 0; p < kKmPoints; ++p) {
        int hs = 0, ls = 0;
#pragma unroll
        for (int w = 0; w < DW; ++w) {
          hs = __builtin_amdgcn_sdot4(x[p][w], cw[c][w], hs, false);
          ls = __builtin_amdgcn_sdot4(x[p][w], cw[c][DW + w], ls, false);
        }
        const int64_t key = cn[c] - 512 * ((int64_t)hs * 256 + ls);
        if (key < best[p]) {
          best[p] = key;
          bi[p] = c0 + c;
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kKmPoints; ++p) {
    const long pt = base + tid + 256 * p;
    if (pt >= n) continue;
    if (prev && changed && prev[pt] != bi[p]) atomicAdd(changed, 1u);
    assign[pt] = bi[p];
  }
}

__global__ void __launch_bounds__(256) k_km_zero(uint64_t* __restrict__ p, long cnt) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < cnt) p[g] = 0;
}

// Thread per (point, coordinate): exact sums and counts of every cluster
// (two's-complement 64-bit atomics).  Assignments outside [0, k) are skipped.
__global__ void __launch_bounds__(256)
k_km_accum(const int8_t* __restrict__ X, long n, int d, const int32_t* __restrict__ assign,
           int k, uint64_t* __restrict__ sums, uint64_t* __restrict__ counts) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * d) return;
  const long pt = g / d;
  const int i = (int)(g % d);
  const int a = assign[pt];
  if (a < 0 || a >= k) return;
  atomicAdd((unsigned long long*)&sums[(size_t)a * d + i],
            (unsigned long long)(int64_t)X[pt * d + i]);
  if (i == 0) atomicAdd((unsigned long long*)&counts[a], 1ull);
}

// Thread per (centre, coordinate): C = floor((2^9 S + n) / (2 n)) for n > 0.
__global__ void __launch_bounds__(256)
k_km_centers(const uint64_t* __restrict__ sums, const uint64_t* __restrict__ counts, int k,
             int d, int32_t* __restrict__ C) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)k * d) return;
  const int j = (int)(g / d);
  const int64_t cnt = (int64_t)counts[j];
  if (cnt == 0) return;
  const int64_t num = (int64_t)sums[g] * 512 + cnt, den = 2 * cnt;
  int64_t q = num / den;
  if (num % den != 0 && num < 0) q -= 1;  // floor
  C[g] = (int32_t)q;
}

// Initial centres: C_j = 2^8 x_{idx[j]}.
__global__ void __launch_bounds__(256)
k_km_init(const int8_t* __restrict__ X, long n, int d, const int64_t* __restrict__ idx, int k,
          int32_t* __restrict__ C, uint32_t* __restrict__ bad) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long)k * d) return;
  const int j = (int)(g / d), i = (int)(g % d);
  long p = idx[j];
  if (p < 0 || p >= n) {
    if (i == 0) atomicOr(bad, 1u);
    p = 0;
  }
  C[g] = 256 * (int32_t)X[p * d + i];
}

int km_words(int d) { return (d + 3) / 4; }

size_t km_workspace(int k, int d) {
  const size_t dw = km_words(d) <= 8 ? 8 : (size_t)(km_words(d) + 7) / 8 * 8;
  return (size_t)k * 2 * dw * 4 + (size_t)k * 8 + (size_t)k * d * 8 + (size_t)k * 8 + 256;
}

static int km_dw(int d) {
  const int w = km_words(d);
  return w <= 8 ? 8 : (w + 7) / 8 * 8;  // 8, 16, ..., 64
}

hipError_t launch_km_init(const int8_t* X, long n, int d, const int64_t* idx, int k, int32_t* C,
                          uint32_t* bad, hipStream_t st) {
  const long t = (long)k * d;
  hipLaunchKernelGGL(k_km_init, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, X, n, d, idx,
                     k, C, bad);
  return hipGetLastError();
}

hipError_t launch_km_assign(const int8_t* X, long n, int d, const int32_t* C, int k,
                            const int32_t* prev, int32_t* assign, uint32_t* changed, void* ws,
                            hipStream_t st) {
  const int dw = km_dw(d);
  int32_t* packed = (int32_t*)ws;
  int64_t* cnorm = (int64_t*)((char*)ws + (size_t)k * 2 * dw * 4);
  hipLaunchKernelGGL(k_km_pack, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, st, C, k, d, dw,
                     packed, cnorm);
  const unsigned grid = (unsigned)((n + 256 * kKmPoints - 1) / (256 * kKmPoints));
  switch (dw) {
#define SANNS_KM(DWV)                                                                       \
  case DWV:                                                                                 \
    hipLaunchKernelGGL(k_km_assign<DWV>, dim3(grid), dim3(256), 0, st, X, n, d, packed, cnorm, \
                       k, prev, assign, changed);                                           \
    break;
    SANNS_KM(8) SANNS_KM(16) SANNS_KM(24) SANNS_KM(32) SANNS_KM(40) SANNS_KM(48) SANNS_KM(56)
    SANNS_KM(64)
#undef SANNS_KM
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_km_update(const int8_t* X, long n, int d, const int32_t* assign, int k,
                            int32_t* C, int64_t* counts_out, void* ws, hipStream_t st) {
  const int dw = km_dw(d);
  uint64_t* sums = (uint64_t*)((char*)ws + (size_t)k * 2 * dw * 4 + (size_t)k * 8);
  uint64_t* counts = sums + (size_t)k * d;
  const long zc = (long)k * d + k;
  hipLaunchKernelGGL(k_km_zero, dim3((unsigned)((zc + 255) / 256)), dim3(256), 0, st, sums, zc);
  const long t = n * d;
  if (t > 0)
    hipLaunchKernelGGL(k_km_accum, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, X, n, d,
                       assign, k, sums, counts);
  const long tc = (long)k * d;
  hipLaunchKernelGGL(k_km_centers, dim3((unsigned)((tc + 255) / 256)), dim3(256), 0, st, sums,
                     counts, k, d, C);
  if (counts_out)
    (void)hipMemcpyAsync(counts_out, counts, (size_t)k * 8, hipMemcpyDeviceToDevice, st);
  return hipGetLastError();
}

}  // namespace sanns
