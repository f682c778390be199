// Shared device-side definitions of the VALMOD HIP implementation (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace valmod {

constexpr int kWave = 64;
constexpr int kIdxBits = 22;  // candidate index bits in a packed (distance, index) key
constexpr uint64_t kIdxMask = (uint64_t(1) << kIdxBits) - 1;
constexpr uint64_t kEmptyKey = ~uint64_t(0);
constexpr int64_t kPad = 4096;  // zero padding after every per-window array

// Packed key of a (correlation, candidate) pair, ordered like the z-normalised
// distance sqrt(2L(1 - rho)) (Eq. 6) and then by candidate index, so an
// unsigned 64-bit min selects the nearest neighbour with ties to the smaller
// index. The distance part keeps the top 42 bits of the double 1 - rho in
// [0, 2] (30 mantissa bits): two candidates that share it differ by less than
// 1e-9 in d / sqrt(L).
__device__ __forceinline__ uint64_t make_key(double rho, int64_t cand) {
  double u = 1.0 - rho;
  u = u > 0.0 ? u : 0.0;  // also maps -0.0 to +0.0
  u = u < 2.0 ? u : 2.0;
  uint64_t bits = (uint64_t)__double_as_longlong(u);
  return ((bits >> kIdxBits) << kIdxBits) | (uint64_t)cand;
}

// Smallest correlation a candidate can have and still produce a key <= `key`,
// lowered by a margin that covers the rounding of 1 - rho.
__device__ __forceinline__ double key_threshold(uint64_t key) {
  if (key == kEmptyKey) return -2.0;
  uint64_t q = key >> kIdxBits;
  double u_hi = __longlong_as_double((long long)((q + 1) << kIdxBits));
  return (1.0 - u_hi) - 4.0e-16;
}

__device__ __forceinline__ int64_t key_cand(uint64_t key) { return (int64_t)(key & kIdxMask); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl_xor((int)lo, m, kWave);
  hi = (uint32_t)__shfl_xor((int)hi, m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int lane) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl((int)lo, lane, kWave);
  hi = (uint32_t)__shfl((int)hi, lane, kWave);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = shfl_xor_u64(v, m);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int m = kWave / 2; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, kWave));
  return v;
}
__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
  for (int m = kWave / 2; m >= 1; m >>= 1) v = fmin(v, __shfl_xor(v, m, kWave));
  return v;
}

__device__ __forceinline__ int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

__host__ __device__ __forceinline__ int64_t excl_zone(int64_t L, int64_t den) {
  return (L + den - 1) / den;
}

// Anchored cross sums formed directly: S[q] = sum_{k<L} (x_{i0+k} - x_{i0}) (x_{c0+q+k} - x_{c0+q})
// for the K consecutive windows c0 + q. The lane's K windows share a register
// window of K values that slides by one element per k; every load is issued one
// block of K steps before its use (the window's entering values and the row
// values of the next block), so the steps do not wait on memory. Reads reach
// x_{c0 + L + 3K} and x_{i0 + L + 2K} (inside the series padding).
template <int K>
__device__ __forceinline__ void direct_sums_ahead(const double* __restrict__ xs, int64_t i0, int64_t c0, int L,
                                                  double* S) {
  const double xi = xs[i0];
  const double* xc = xs + c0;
  const double* xr = xs + i0;
  double base[K], w[K], nx[K], r[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    base[q] = xc[q];
    w[q] = base[q];
    nx[q] = xc[K + q];  // enters slot q during the first block
    r[q] = xr[q];
    S[q] = 0.0;
  }
  for (int kb = 0; kb < L; kb += K) {
    double nn[K], rn[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      nn[u] = xc[2 * K + kb + u];  // enters during the next block
      rn[u] = xr[K + kb + u];
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
      if (kb + u >= L) break;
      const double rv = r[u] - xi;
#pragma unroll
      for (int q = 0; q < K; ++q) S[q] = fma(rv, w[(q + u) % K] - base[q], S[q]);
      w[u] = nx[u];  // the slot of x_{c0 + kb + u} takes x_{c0 + K + kb + u}
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
      nx[u] = nn[u];
      r[u] = rn[u];
    }
  }
}

}  // namespace valmod
