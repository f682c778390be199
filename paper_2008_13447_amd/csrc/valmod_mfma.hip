// Hankel-block contractions on FP64 matrix cores (gfx950 MFMA): the dense
// dot-product blocks of the VALMOD hot path.
//
// Both the anchor table of the diagonal pass (the first-row dot products of
// Alg. ComputeMatrixProfile, one per segment start and diagonal) and the exact
// row recompute of the windows whose bound test fails (the non-valid distance
// profiles of Alg. ComputeSubMP) are blocks of one product
//   M[r][j] = sum_{k<L} (x_{a_r + k} - x_{a_r}) (x_{j + k} - x_{j})
// of a set of row windows a_r with a range of consecutive column windows j: a
// (rows x L) by (L x columns) contraction whose right operand is a Hankel matrix
// of the series. It is dense, so it runs on v_mfma_f64_16x16x4f64: one wavefront
// owns 16 rows and 64 consecutive columns (four 16 x 16 accumulators) and walks k
// four terms at a time. Operand layout of the instruction: A (16 x 4) lane l
// holds row l % 16, term l / 16; B (4 x 16) lane l holds column l % 16, term
// l / 16; the 16 x 16 result gives lane l column l % 16 and, in its register v =
// 0..3, row 4 v + l / 16 (measured on gfx950). Terms past L are zero. The window values are excursions from each
// window's first point, as in the VALU kernels, so no large-offset
// cancellation occurs; the sum's rounding is covered by the same bound as a
// direct sum of L terms in any order.
#include "valmod_common.h"
#include "valmod_kernels.h"

#include <math.h>

namespace valmod {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTileCols = 64;  // columns per wavefront (four 16-column accumulators)
constexpr int kNB = kTileCols / 16;

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// acc[c] += the 16 x 16 block of rows `ra` (this lane's row start, one per
// l % 16) and columns j0 + 16 c + (l % 16), summed over k < L. The operands of
// a group of four terms are loaded two groups before their products run, and
// every load is unconditional (a term past L is zeroed after its load), so no
// load waits inside a branch. Reads reach at most L + 10 past a window's start
// (the row's and the last column's), inside the series' zero padding.
__device__ __forceinline__ void hankel_block(const double* __restrict__ xs, int64_t ra, int64_t j0, int L,
                                             f64x4 acc[kNB]) {
  const int l = threadIdx.x & (kWave - 1);
  const int kk = l >> 4;
  const int64_t jb = j0 + (l & 15);
  const double xa0 = xs[ra];
  double xb0[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) xb0[c] = xs[jb + 16 * c];
  // two groups in flight: terms k0 + kk (set 0) and k0 + 4 + kk (set 1)
  double a0 = xs[ra + kk], a1 = xs[ra + 4 + kk];
  double b0[kNB], b1[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) {
    b0[c] = xs[jb + 16 * c + kk];
    b1[c] = xs[jb + 16 * c + 4 + kk];
  }
  auto group = [&](int k0, double& an, double* bn) {
    const bool in = k0 + kk < L;
    const double a = in ? an - xa0 : 0.0;
    double b[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) b[c] = in ? bn[c] - xb0[c] : 0.0;
    const int kn = k0 + 8 + kk;  // this set's next group
    an = xs[ra + kn];
#pragma unroll
    for (int c = 0; c < kNB; ++c) bn[c] = xs[jb + 16 * c + kn];
#pragma unroll
    for (int c = 0; c < kNB; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[c], acc[c], 0, 0, 0);
  };
  for (int k0 = 0; k0 < L; k0 += 8) {
    group(k0, a0, b0);
    if (k0 + 4 < L) group(k0 + 4, a1, b1);
  }
}

// Anchor table at length L: anc[s * stride + d] = M[s][s H + dstart + d] for
// every segment s and diagonal index d < ncols whose column j has a window
// (j + L <= n). Grid: x = chunks of 64 columns, y = groups of 16 segments;
// chunks entirely below the first segment's band exit at once.
__global__ __launch_bounds__(kWave) void k_anchor_mfma(const double* __restrict__ xs, int64_t n, int L, int64_t H,
                                                       int64_t dstart, int64_t segs, int64_t stride, int64_t ncols,
                                                       double* __restrict__ anc) {
  const int64_t s0 = (int64_t)blockIdx.y * 16;
  const int64_t j0 = (int64_t)blockIdx.x * kTileCols;
  const int64_t N = n - L + 1;
  const int64_t s_last = s0 + 15 < segs - 1 ? s0 + 15 : segs - 1;
  // the block's columns must meet some segment's band [s H + dstart, s H + dstart + ncols) below N
  if (j0 >= N || j0 + kTileCols <= s0 * H + dstart || j0 >= s_last * H + dstart + ncols) return;
  const int l = threadIdx.x & (kWave - 1);
  const int64_t sr = s0 + (l & 15);
  const int64_t ra = (sr < segs ? sr : segs - 1) * H;  // rows past the last segment repeat it (not stored)
  f64x4 acc[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
  hankel_block(xs, ra, j0, L, acc);
#pragma unroll
  for (int c = 0; c < kNB; ++c) {
    const int64_t j = j0 + 16 * c + (l & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t s = s0 + 4 * v + (l >> 4);
      const int64_t d = j - s * H - dstart;
      if (s < segs && d >= 0 && d < ncols && j < N) anc[s * stride + d] = acc[c][v];
    }
  }
}

// Exact row recompute: for the listed owners (16 per wavefront, a grid-stride
// walk over the device-side list) and chunks of 64 candidates (a grid-stride
// walk too, so that the grid stays small when the list is short or empty), the
// best key (correlation, candidate) over the eligible candidates, merged into
// the owner's key by a 64-bit atomic min (the listing kernel set it to empty).
//
// The same kernel serves the rounds of the top-m recompute: with m > 1 the
// owner's result goes to out[o * m + j] and only keys strictly above its key of
// round j - 1 (out[o * m + j - 1]) take part; an owner whose previous round found
// nothing is skipped.
__global__ __launch_bounds__(kWave) void k_recompute_mfma(const double* __restrict__ xs, const double* __restrict__ A,
                                                          const double* __restrict__ invn,
                                                          const uint8_t* __restrict__ flat,
                                                          const int32_t* __restrict__ list,
                                                          const unsigned long long* __restrict__ nlist, int64_t N,
                                                          int L, int64_t e, int m, int jr, uint64_t* __restrict__ out) {
  const int64_t count = (int64_t)*nlist;
  const int l = threadIdx.x & (kWave - 1);
  for (int64_t j0 = (int64_t)blockIdx.x * kTileCols; j0 < N; j0 += (int64_t)gridDim.x * kTileCols)
  for (int64_t rb = (int64_t)blockIdx.y * 16; rb < count; rb += (int64_t)gridDim.y * 16) {
    const int64_t ri = rb + (l & 15);
    const int64_t ra = list[ri < count ? ri : count - 1];  // rows past the list repeat its last owner
    f64x4 acc[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
    hankel_block(xs, ra, j0, L, acc);
    // this lane's results: rows 4 v + l / 16, columns j0 + 16 c + l % 16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t rr = rb + 4 * v + (l >> 4);
      const bool live = rr < count;
      const int64_t o = live ? list[rr] : 0;
      const uint64_t floor_key = (live && jr > 0) ? out[o * m + jr - 1] : 0;
      const bool own = live && !flat[o] && (jr == 0 || floor_key != kEmptyKey);
      const double Ao = own ? A[o] : 0.0, io = own ? invn[o] : 0.0;
      uint64_t kb = kEmptyKey;
#pragma unroll
      for (int c = 0; c < kNB; ++c) {
        const int64_t j = j0 + 16 * c + (l & 15);
        if (own && j < N && iabs64(j - o) > e && !flat[j]) {
          const double rho = (acc[c][v] - Ao * A[j] / (double)L) * io * invn[j];
          const uint64_t key = make_key(rho, j);
          if (jr == 0 || key > floor_key) kb = key < kb ? key : kb;
        }
      }
      // min over the 16 lanes that share this row (same l / 16)
#pragma unroll
      for (int m = 8; m >= 1; m >>= 1) {
        const uint64_t other = shfl_xor_u64(kb, m);
        kb = other < kb ? other : kb;
      }
      if ((l & 15) == 0 && live && kb != kEmptyKey)
        atomicMin((unsigned long long*)&out[o * m + jr], (unsigned long long)kb);
    }
  }
}

}  // namespace

hipError_t launch_anchor_mfma(const double* xs, int64_t n, int L, int64_t H, int64_t dstart, int64_t segs,
                              int64_t stride, int64_t ncols, double* anc, hipStream_t st) {
  const int64_t N = n - L + 1;
  if (segs <= 0 || ncols <= 0 || N <= 0) return hipSuccess;
  const dim3 grid(blocks_for(N, kTileCols), (unsigned)((segs + 15) / 16));
  k_anchor_mfma<<<grid, kWave, 0, st>>>(xs, n, L, H, dstart, segs, stride, ncols, anc);
  return hipGetLastError();
}

hipError_t launch_recompute_mfma(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                 const int32_t* list, const unsigned long long* nlist, int64_t max_listed, int64_t N,
                                 int L, int64_t e, uint64_t* best, hipStream_t st) {
  return launch_recompute_round_mfma(xs, A, invn, flat, list, nlist, max_listed, N, L, e, 1, 0, best, st);
}

hipError_t launch_recompute_round_mfma(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                       const int32_t* list, const unsigned long long* nlist, int64_t max_listed,
                                       int64_t N, int L, int64_t e, int m, int jr, uint64_t* out, hipStream_t st) {
  if (max_listed <= 0 || N <= 0) return hipSuccess;
  if (m < 1 || jr < 0 || jr >= m) return hipErrorInvalidValue;
  const int64_t groups = (max_listed + 15) / 16;
  const unsigned chunks = blocks_for(N, kTileCols);
  const dim3 grid(chunks < 2048 ? chunks : 2048, (unsigned)(groups < 16 ? groups : 16));
  k_recompute_mfma<<<grid, kWave, 0, st>>>(xs, A, invn, flat, list, nlist, N, L, e, m, jr, out);
  return hipGetLastError();
}

}  // namespace valmod
