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

// --------------------------------------------------------------------------
// Rounding bounds, in correlation units (rho = C / (sw_i sw_j), sw = sigma sqrt(L)).
//
// Direct anchored sums S = sum_{k<L} a_k b_k with a_k = x_{o+k} - x_o: an FMA
// chain (or one FMA per length when grown) errs by at most L u sum |a_k b_k|
// <= L u |a| |b| (u = 2^-53), and |a|^2 = L sigma^2 + L (mu - x_o)^2 <=
// L (L + 1) sigma^2, so |a| |b| <= (L + 1) sw_o sw_c. The conversion to the
// co-moment (S - A_o A_c / L, |A_o A_c| / L <= L sw_o sw_c) and the
// normalisation add a few units more: (L + 1)(L + 2) 2^-52 covers all of it.
__host__ __device__ __forceinline__ double direct_bound(int L) {
  return (double)(L + 1) * (double)(L + 2) * 2.220446049250313e-16;
}

// The diagonal recurrence over a work item of H rows, in a precision with unit
// roundoff eps: each step adds two rounded FMAs on |C| <= sw_i sw_j, the inputs
// df, dg carry one rounding each, and the start and the normalisation a few
// more. The means inside dg = (x_{i+L} - mu_{i+1}) + (x_i - mu_i) are FP64 values
// near the series level, so dg also carries their absolute rounding, up to
// 2 u max|mu| (u = 2^-53), which each step multiplies by |df|. With
// Phi = (max sw / min sw)_rows (max sw / min sw)_cols,
// Psi = (max|df|_rows max|dg|_cols + max|dg|_rows max|df|_cols) / (min sw_rows min sw_cols) and
// Xi = (max|df|_rows + max|df|_cols) max|mu| / (min sw_rows min sw_cols)
// over the item's windows, the first-order error of rho after r <= H steps is
// at most eps [(2H + 1) Phi + 4 H Psi + 4] + 2 u H Xi; the bound doubles it for
// the higher-order terms and adds the error of the FP64 anchor it starts from.
__host__ __device__ __forceinline__ double recurrence_bound(double eps, double H, double phi, double psi, double xi,
                                                           int L) {
  return 2.0 * (eps * ((2.0 * H + 1.0) * phi + 4.0 * H * psi + 4.0) + 2.0 * 1.1102230246251565e-16 * H * xi) +
         direct_bound(L);
}
constexpr double kEps32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kEps64 = 1.1102230246251565e-16;   // 2^-53
// the FP32 filter compares the rounded difference rho - threshold (|.| < 4)
// with -delta: one more FP32 ulp at magnitude 2..4
constexpr double kFilter32 = 2.384185791015625e-07;  // 2^-22

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
