// Diagonal pass of the VALMOD hot path (gfx950): anchor table and the
// co-moment recurrence over the upper triangle of the distance matrix.
#include "valmod_common.h"
#include "valmod_kernels.h"

#include <hip/hip_ext.h>
#include <math.h>
#include <type_traits>

namespace valmod {

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// --------------------------------------------------------------------------
// Anchor table of the diagonal pass (the first-row dot products of
// Alg. ComputeMatrixProfile, one per work item and diagonal):
//   S(i0, i0 + d) = sum_{k<L} (x_{i0+k} - x_{i0}) (x_{i0+d+k} - x_{i0+d})
// for every segment start row i0 = seg * H and diagonal d >= dstart. Values
// are excursions from each window's first point (no large-offset
// cancellation); the pass turns them into co-moments with C = S - A_i A_j / L.
// k_anchor_init forms them directly (L FMAs each); when the length grows by one
// the single new term is added, so later lengths cost O(1) per anchor: by the
// last pass of a length as it reads the anchors, or by k_anchor_grow when a
// length runs no pass.
__global__ void k_anchor_init(const double* __restrict__ xs, int64_t n, int L, int64_t H, int64_t dstart,
                              int64_t stride, int64_t ncols, double* __restrict__ anc) {
  const int64_t seg = blockIdx.y;
  const int64_t dd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dd >= ncols) return;
  const int64_t i0 = seg * H;
  const int64_t j0 = i0 + dstart + dd;
  double acc = 0.0;
  if (j0 + L <= n) {
    const double xi = xs[i0], xj = xs[j0];
    for (int k = 1; k < L; ++k) acc = fma(xs[i0 + k] - xi, xs[j0 + k] - xj, acc);
  }
  anc[seg * stride + dd] = acc;
}

__global__ void k_anchor_grow(const double* __restrict__ xs, int64_t n, int L, int64_t H, int64_t dstart,
                              int64_t stride, int64_t ncols, double* __restrict__ anc) {
  // L is the new length: adds the term k = L - 1
  const int64_t seg = blockIdx.y;
  const int64_t dd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dd >= ncols) return;
  const int64_t i0 = seg * H;
  const int64_t j0 = i0 + dstart + dd;
  if (j0 + L > n) return;
  anc[seg * stride + dd] = fma(xs[i0 + L - 1] - xs[i0], xs[j0 + L - 1] - xs[j0], anc[seg * stride + dd]);
}

// --------------------------------------------------------------------------
// Diagonal pass (Alg. ComputeMatrixProfile).
//
// One wavefront owns a band of 64*K adjacent diagonals d = j - i (K per lane)
// and a segment of H rows. Each lane runs the co-moment recurrence of its K
// diagonals in registers, from an FP64 anchor computed directly at the
// segment's first row. Every cell (i, j) is seen once and serves two owners by
// symmetry: row owner i (candidate j) and column owner j (candidate i).
//
// The per-cell work is the two-FMA update and a test against both owners'
// thresholds (correlation units): the cell can matter only if
// rho = C invn_i invn_j >= min(thr_i, thr_j), with invn = 1 / (sigma sqrt L).
// The FP32 pass takes the largest C invn_j over the lane's K cells, scales it by
// the row's inverse norm and raises it by the item's rounding bound (one fma),
// and compares it with the lane's threshold: the minimum of the row's threshold
// and those of the column slots the block has used (a superset of the cells that
// pass per cell, at K multiplies and a max tree per step instead of K
// multiplies, K minimums, K fmas and K compares). The FP64 pass takes the same
// test. A step whose wavefront has a passing cell goes to a slow path that
// evaluates rho per cell and applies the mode's action:
//   MODE_MP     : running best of each owner as a packed (distance, index) key
//                 updated by 64-bit atomic min; thr = the running best's bound.
//   MODE_APPEND : thr is a fixed per-owner threshold; every candidate with
//                 rho >= thr is appended to the owner's list (the partial
//                 distance profile of Alg. ComputeMatrixProfile, collected as all
//                 candidates above a threshold instead of a heap insert per cell).
// Column data slide through a per-lane register window of K columns (one new
// column per row, 32-bit offsets off a uniform base); row data are wave-uniform
// scalar loads, once per K rows.
enum { MODE_MP = 0, MODE_APPEND = 1 };

struct PassArgs {
  double* thr;         // per-owner threshold (correlation units); MODE_MP updates it
  uint64_t* best;      // MODE_MP: packed best key per owner
  uint32_t* cnt;       // MODE_APPEND: candidates appended per owner
  int32_t* buf;        // MODE_APPEND: owner-major candidate lists
  int64_t cap;         // MODE_APPEND: list capacity per owner
  unsigned long long* events;  // [0] wave-steps that took the slow path, [1] queue entries
  const int32_t* items;        // optional list of work items (seg * bands + band); null: the whole grid
  const unsigned long long* nitems;  // number of listed items (device count; the grid may be larger)
  const float* delta;          // bound of |rho computed - rho| per work item (null: none)
  float delta_max;             // items with a larger bound are skipped (left to the FP64 kernel)
  int64_t anc_stride;  // anchor-table row length (diagonals per segment row)
  double* anc_next;    // optional: the item's anchors are moved on to length L + 1 in place
  int64_t bands;       // bands of the grid (decodes item ids)
  int64_t N, e, H, dstart;
  int L;
};

template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t off) {
  return *(const T*)((const char*)base + off);
}

// Wide per-lane loads of `n` consecutive elements (lanes read adjacent ranges,
// so a wavefront reads one contiguous block).
template <int n>
__device__ __forceinline__ void load_run(const double* p, double* dst) {
#pragma unroll
  for (int u = 0; u < n; u += 2) {
    const double2 v = *(const double2*)(p + u);
    dst[u] = v.x;
    dst[u + 1] = v.y;
  }
}
template <int n>
__device__ __forceinline__ void load_run(const float* p, float* dst) {
  static_assert(n % 2 == 0, "float runs are loaded 4 (or 2) at a time");
  if (n % 4 == 0) {
#pragma unroll
    for (int u = 0; u < n; u += 4) {
      const float4 v = *(const float4*)(p + u);
      dst[u] = v.x;
      dst[u + 1] = v.y;
      dst[u + 2] = v.z;
      dst[u + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int u = 0; u < n; u += 2) {
      const float2 v = *(const float2*)(p + u);
      dst[u] = v.x;
      dst[u + 1] = v.y;
    }
  }
}

// Per-wavefront LDS queue of slow-path results. The step loop issues no global
// writes or atomics (on gfx9 they share the load counter with the prefetch
// loads, and a write inside a data-dependent branch makes every later wait
// drain all prefetches); the queue is flushed to global memory when it could
// overflow at the next step and at the end of the work item.
// Queue capacity of a wavefront: 2 * 64 * K entries (a matrix-profile step adds
// at most 64 K + 1, a collecting step at most 64).
template <int K>
struct PassQueue {
  static constexpr int size = 2 * kWave * K;
};

// min of two thresholds (never NaN) without the IEEE quieting of the operands
// that fmin() implies.
__device__ __forceinline__ double vmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float vmin(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// One more term of the anchor sums of an item (lane t: diagonals d0 + K t + q):
// the table then holds length L + 1 for the diagonals with a window there
// (j < N - 1). Every anchor belongs to one item and is read only by it, so
// the entries are still those of length L. Kept out of line so that the
// addresses it needs are not held in registers across the rows.
template <int K>
__device__ __attribute__((noinline)) void grow_anchors(const double* __restrict__ xs, double* __restrict__ row,
                                                       int64_t i0, int64_t d0, int64_t N, int L) {
  const int64_t dl = d0 + (int64_t)K * threadIdx.x;
  double* an = row + dl;
  double S[K], xj[K], xjl[K];
  load_run<K>(an, S);
  load_run<K>(xs + i0 + dl, xj);
  load_run<K>(xs + i0 + dl + L, xjl);
  const double xr = xs[i0 + L] - xs[i0];
#pragma unroll
  for (int q = 0; q < K; ++q)
    if (i0 + dl + q < N - 1) an[q] = fma(xr, xjl[q] - xj[q], S[q]);
}

// LIST = false: one work item per workgroup over the whole grid. LIST = true:
// the workgroups walk the device-side item list (item w, w + gridDim.x, ...),
// so the grid stays small whatever the list length.
template <typename T, int K, int MODE, bool LIST>
__global__ __launch_bounds__(kWave) void k_pass(const T* __restrict__ g_df, const T* __restrict__ g_dg,
                                                const T* __restrict__ g_invn, const T* __restrict__ g_thr,
                                                const double* __restrict__ g_xs, const double* __restrict__ g_anc,
                                                const double* __restrict__ g_A, PassArgs a) {
  // g_thr aliases the threshold array this kernel updates in MODE_MP: reads
  // through it may return older values, which only loosens the filter.
  static_assert(K % 4 == 0, "run loads need K multiple of 4");
  constexpr int64_t BW = (int64_t)kWave * K;  // diagonals per band
  constexpr int HK = K / 2;
  constexpr int kQueue = PassQueue<K>::size;
  using QVal = typename std::conditional<MODE == MODE_MP, uint64_t, uint32_t>::type;
  __shared__ int32_t q_owner[kQueue];
  __shared__ QVal q_val[kQueue];  // MODE_MP: packed key; MODE_APPEND: candidate index
  const int t = threadIdx.x;
  const int64_t N = a.N;
  const int64_t nlist = LIST ? (int64_t)*a.nitems : 0;
  int64_t w = blockIdx.x;
  for (;;) {
  {  // one work item (a skipped item jumps to `next`)
  int64_t seg = blockIdx.x, band = blockIdx.y;
  if (LIST) {
    if (w >= nlist) return;
    const int64_t id = a.items[w];
    seg = id / a.bands;
    band = id % a.bands;
  } else if (a.items) {  // (not used: listed items take LIST = true)
    if ((unsigned long long)blockIdx.x >= *a.nitems) return;
    const int64_t id = a.items[blockIdx.x];
    seg = id / a.bands;
    band = id % a.bands;
  }
  const int64_t d0 = a.dstart + band * BW;
  if (d0 > N - 1) goto next;
  const int64_t i0 = seg * a.H;
  const int64_t rowEnd = N - d0;
  if (i0 >= rowEnd) goto next;
  // rigorous bound of the rounding of rho over this item (collecting passes)
  T delta = (T)0;
  if (a.delta) {
    const float dl_ = a.delta[seg * a.bands + band];
    if (!(dl_ <= a.delta_max)) goto next;  // left to the FP64 kernel
    delta = (T)dl_;
  }
  const int rows = (int)((i0 + a.H < rowEnd ? i0 + a.H : rowEnd) - i0);
  // the bound in a vector register: the filter's fma then reads one scalar (the
  // row's inverse norm) instead of two, which would need a move at every step
  T delta_v = delta;
  if constexpr (sizeof(T) == 4) asm volatile("v_mov_b32 %0, %1" : "=v"(delta_v) : "s"(delta));
  const int64_t dl = d0 + (int64_t)K * t;

  // co-moments at row i0 from FP64 anchors: C = S - A_i A_j / L
  T C[K];
  {
    double S[K], Aj[K];
    if (g_anc)
      load_run<K>(g_anc + seg * a.anc_stride + (dl - a.dstart), S);
    else
      direct_sums_ahead<K>(g_xs, i0, i0 + dl, a.L, S);
    load_run<K>(g_A + i0 + dl, Aj);
    const double Ai = g_A[i0] / (double)a.L;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int64_t j = i0 + dl + q;
      C[q] = (dl + q > a.e && j < N) ? (T)(S[q] - Ai * Aj[q]) : (T)-INFINITY;  // trivial or past the end
    }
  }

  // Column window: at step u of a block, slot s holds column i + dl + ((s - u) mod K).
  // Two register sets X and Y alternate by block: during a block whose slots
  // start in set P, slot s moves to set Q (holding the column that enters) at
  // step s, and the freed entries of P receive the next block's entering
  // columns, a half block at a time. No register copies are needed.
  T Xdf[K], Xdg[K], Xinv[K], Xthr[K];
  T Ydf[K], Ydg[K], Yinv[K], Ythr[K];
  {
    const int64_t c0 = i0 + dl;
    load_run<K>(g_df + c0, Xdf);
    load_run<K>(g_dg + c0, Xdg);
    load_run<K>(g_invn + c0, Xinv);
    load_run<K>(g_thr + c0, Xthr);
    load_run<K>(g_df + c0 + K, Ydf);
    load_run<K>(g_dg + c0 + K, Ydg);
    load_run<K>(g_invn + c0 + K, Yinv);
    load_run<K>(g_thr + c0 + K, Ythr);
  }
  int qn = 0;  // queue fill (wave-uniform)
  unsigned long long ev_steps = 0;

  // MODE_MP entries: (owner, packed key). MODE_APPEND entries: one per lane and
  // step, (row i, lane t | cell mask << 6): bit q of the mask appends row i to
  // column owner i + d0 + K t + q, bit K + q appends that column to row owner i.
  auto flush = [&]() {
    __syncthreads();
    unsigned long long hits = 0;
    for (int b = 0; b < qn; b += kWave) {
      if (b + t < qn) {
        const int32_t own = q_owner[b + t];
        const uint64_t v = q_val[b + t];
        if (MODE == MODE_MP) {
          atomicMin((unsigned long long*)&a.best[own], (unsigned long long)v);
          const double nt = key_threshold(v);
          if (nt > a.thr[own]) a.thr[own] = nt;  // racy but every stored value is a real candidate's bound
        } else {
          const int64_t j0 = (int64_t)own + d0 + (int64_t)K * (int64_t)(v & 63u);
          uint32_t m = (uint32_t)(v >> 6);
          while (m) {
            const int q = __ffs(m) - 1;
            m &= m - 1;
            const bool col = q < K;
            const int64_t j = j0 + (col ? q : q - K);
            const int64_t o = col ? j : (int64_t)own;
            const uint32_t pos = atomicAdd(&a.cnt[o], 1u);
            if ((int64_t)pos < a.cap) a.buf[o * a.cap + pos] = (int32_t)(col ? (int64_t)own : j);
            hits += 1;
          }
        }
      }
    }
    if (MODE == MODE_MP) {
      if (a.events && t == 0) atomicAdd(&a.events[1], (unsigned long long)qn);
    } else if (a.events) {
#pragma unroll
      for (int m = kWave / 2; m >= 1; m >>= 1) hits += shfl_xor_u64(hits, m);
      if (t == 0 && hits) atomicAdd(&a.events[1], hits);
    }
    __syncthreads();
    qn = 0;
  };
  // append the lanes of mask m (this lane: `want`) to the queue
  auto push_m = [&](uint64_t m, bool want, int32_t owner, uint64_t val) {
    if (!m) return;
    if (want) {
      const int pos = qn + __popcll(m & ((uint64_t(1) << t) - 1));
      q_owner[pos] = owner;
      q_val[pos] = (QVal)val;
    }
    qn += __popcll(m);
  };
  auto push = [&](bool want, int32_t owner, uint64_t val) { push_m(__ballot(want), want, owner, val); };

  // one block of K rows starting at row ib; slots start in P and move to Q
  auto block = [&](int64_t ib, T* Pdf, T* Pdg, T* Pinv, T* Pthr, T* Qdf, T* Qdg, T* Qinv, T* Qthr) {
    T rdf[K], rdg[K], rinv[K], rthr[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      rdf[u] = g_df[ib + u];
      rdg[u] = g_dg[ib + u];
      rinv[u] = g_invn[ib + u];
      rthr[u] = g_thr[ib + u];
    }
    const int64_t cn = ib + dl + 2 * K;  // first column entering during the next block
    // FP32 filter threshold of the lane: the running minimum of the thresholds of
    // the column slots the block has used so far (the current set at its start,
    // then each column as it enters), taken with the step's row threshold
    T tcol;
    {
      T m[K];
#pragma unroll
      for (int q = 0; q < K; ++q) m[q] = Pthr[q];
#pragma unroll
      for (int w = 1; w < K; w *= 2)
#pragma unroll
        for (int q = 0; q + w < K; q += 2 * w) {
          if constexpr (sizeof(T) == 4)
            m[q] = __builtin_elementwise_minimum(m[q], m[q + w]);
          else
            m[q] = vmin(m[q], m[q + w]);
        }
      tcol = m[0];
    }
    // Every block runs all K steps: rows past the segment or the series only meet
    // columns past the end (zero inverse norm, padded thresholds), so they never
    // produce a queue entry, and all their reads stay inside the zero padding.
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int64_t i = ib + u;
      // the cells of the step against both owners' thresholds, one test per lane
      // (no per-cell mask traffic): the largest C invn_j, scaled by invn_i and
      // raised by the rounding bound with one rounding, against the smallest
      // threshold the lane's cells can have. The thresholds are never NaN (the
      // NaN-propagating minimum is exact here); the max ignores the NaN inverse
      // norms of flat and padded windows in the FP32 copies.
      bool any_pass;
      if constexpr (sizeof(T) == 4) {
        // the largest C invn_j over the lane's cells, scaled by the row's inverse
        // norm and raised by the rounding bound with one rounding (fma), against
        // the lane's threshold: a superset of the cells whose correlation reaches
        // min(thr_i, thr_j) lowered by the bound; the slow path tests each cell
        if (u > 0) tcol = __builtin_elementwise_minimum(tcol, Qthr[u - 1]);  // the column that entered
        T dq[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const int s = (q + u) % K;
          dq[q] = C[q] * (s < u ? Qinv[s] : Pinv[s]);
        }
        T mx;
        if constexpr (K == 8) {  // three-input maxima: 4 instructions for 8 values, 3 deep
          const T m0 = __builtin_fmaxf(__builtin_fmaxf(dq[0], dq[1]), dq[2]);
          const T m1 = __builtin_fmaxf(__builtin_fmaxf(dq[3], dq[4]), dq[5]);
          const T m2 = __builtin_fmaxf(__builtin_fmaxf(dq[6], dq[7]), m0);
          mx = __builtin_fmaxf(m1, m2);
        } else {
#pragma unroll
          for (int w = 1; w < K; w *= 2)  // pairwise, to keep the dependency chain short
#pragma unroll
            for (int q = 0; q + w < K; q += 2 * w) dq[q] = __builtin_fmaxf(dq[q], dq[q + w]);
          mx = dq[0];
        }
        any_pass = __builtin_expect(
            __any(fma(mx, rinv[u], delta_v) >= __builtin_elementwise_minimum(tcol, rthr[u])), 0);
      } else {
        // FP64: the same superset test (delta = 0 in matrix-profile mode, where
        // the slow path raises thresholds during the block: the running minimum
        // taken before only loosens the test)
        if (u > 0) tcol = vmin(tcol, Qthr[u - 1]);
        T dq[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const int s = (q + u) % K;
          dq[q] = C[q] * (s < u ? Qinv[s] : Pinv[s]);
        }
#pragma unroll
        for (int w = 1; w < K; w *= 2)
#pragma unroll
          for (int q = 0; q + w < K; q += 2 * w) dq[q] = __builtin_fmax(dq[q], dq[q + w]);
        any_pass = __builtin_expect(__any(fma(dq[0], rinv[u], delta) >= vmin(tcol, rthr[u])), 0);
      }
      if (MODE == MODE_MP && any_pass) {
        ++ev_steps;
        // at most K column entries per lane and one row entry per step
        if (qn + kWave * K + 1 > kQueue) flush();
        uint64_t rowkey = kEmptyKey;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const int s = (q + u) % K;
          const int64_t j = i + dl + q;
          const T inv = s < u ? Qinv[s] : Pinv[s];
          T& th = s < u ? Qthr[s] : Pthr[s];
          const T rho = (C[q] * inv) * rinv[u];
          const bool ok = j < N && rinv[u] > (T)0 && inv > (T)0;
          const bool col = ok && rho >= th;  // (matrix-profile mode: no rounding bound)
          const uint64_t key = col ? make_key((double)rho, i) : kEmptyKey;
          push(col, (int32_t)j, key);
          if (col) {
            const T nt = (T)key_threshold(key);
            th = nt > th ? nt : th;
          }
          if (ok && rho >= rthr[u]) {
            const uint64_t k2 = make_key((double)rho, j);
            rowkey = k2 < rowkey ? k2 : rowkey;
          }
        }
        if (__any(rowkey != kEmptyKey)) {
          rowkey = wave_min_u64(rowkey);
          push(t == 0, (int32_t)i, rowkey);
        }
      } else if (MODE == MODE_APPEND && any_pass) {
        ++ev_steps;
        // one queue entry per lane with a passing cell: its column and row bits
        uint32_t mask = 0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const int s = (q + u) % K;
          const int64_t j = i + dl + q;
          const T inv = s < u ? Qinv[s] : Pinv[s];
          const T thc = s < u ? Qthr[s] : Pthr[s];
          // FP32: flat and padded windows have a NaN inverse norm, so rho is NaN
          // and fails both tests; FP64: zero inverse norms are tested
          const bool ok = sizeof(T) == 4 || (j < N && rinv[u] > (T)0 && inv > (T)0);
          bool colp, rowp;
          if constexpr (sizeof(T) == 4) {
            // thresholds lowered by the rounding bound (the bound includes the
            // rounding of these differences)
            const T rho = (C[q] * inv) * rinv[u];
            colp = rho >= thc - delta;
            rowp = rho >= rthr[u] - delta;
          } else {
            const T rp = fma(C[q] * inv, rinv[u], delta);  // as in the filter
            colp = rp >= thc;
            rowp = rp >= rthr[u];
          }
          mask |= (ok && colp) ? (1u << q) : 0u;
          mask |= (ok && rowp) ? (1u << (K + q)) : 0u;
        }
        if (qn + kWave > kQueue) flush();
        push(mask != 0, (int32_t)i, (uint64_t)((uint32_t)t | (mask << 6)));
      }
      // advance every diagonal one row: C(i+1, j+1) = C(i, j) + df_i dg_j + df_j dg_i
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int s = (q + u) % K;
        const T cdf = s < u ? Qdf[s] : Pdf[s];
        const T cdg = s < u ? Qdg[s] : Pdg[s];
        C[q] = fma(rdf[u], cdg, C[q]);
        C[q] = fma(cdf, rdg[u], C[q]);
      }
      // slot u now moves to Q (column i + dl + K). Freed P entries take the
      // next block's entering columns, half a block at a time.
      if (u == HK - 1) {
        load_run<HK>(g_df + cn, Pdf);
        load_run<HK>(g_dg + cn, Pdg);
        load_run<HK>(g_invn + cn, Pinv);
        load_run<HK>(g_thr + cn, Pthr);
      } else if (u == K - 1) {
        load_run<HK>(g_df + cn + HK, Pdf + HK);
        load_run<HK>(g_dg + cn + HK, Pdg + HK);
        load_run<HK>(g_invn + cn + HK, Pinv + HK);
        load_run<HK>(g_thr + cn + HK, Pthr + HK);
      }
    }
  };

  for (int sb = 0; sb < rows; sb += 2 * K) {
    block(i0 + sb, Xdf, Xdg, Xinv, Xthr, Ydf, Ydg, Yinv, Ythr);
    if (sb + K < rows) block(i0 + sb + K, Ydf, Ydg, Yinv, Ythr, Xdf, Xdg, Xinv, Xthr);
  }
  if (qn > 0) flush();
  if (a.events && t == 0 && ev_steps) atomicAdd(&a.events[0], ev_steps);
  // after the rows, so that no store precedes the loop's loads
  if (a.anc_next) grow_anchors<K>(g_xs, a.anc_next + seg * a.anc_stride - a.dstart, i0, d0, N, a.L);
  }
  next:
  if (!LIST) return;
  w += gridDim.x;
  }
}

// --------------------------------------------------------------------------
// Rounding bounds of the recurrence per work item (recurrence_bound: H = the
// segment height, Phi and Psi from the per-64-window extrema of sigma sqrt(L),
// |df| and |dg| of the item's rows and columns, flat windows excluded). The
// FP64 bound is always written; it widens the thresholds of the FP64 collecting
// passes, so every candidate whose exact correlation reaches its owner's
// threshold is collected. With delta32, also the FP32 bound (plus one ulp for
// the filter's own difference), and the items whose FP32 bound exceeds the limit
// are listed for the FP64 kernel.
__global__ void k_item_bounds(const float* __restrict__ bsw_max, const float* __restrict__ bsw_min,
                              const float* __restrict__ bdf_max, const float* __restrict__ bdg_max,
                              const float* __restrict__ bmu_max, int64_t nblk,
                              int64_t segs, int64_t bands, int64_t H, int64_t dstart, int64_t BW, int64_t N, int L,
                              float delta_max, float* __restrict__ delta64, float* __restrict__ delta32,
                              int32_t* __restrict__ hard, unsigned long long* __restrict__ nhard) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= segs * bands) return;
  const int64_t seg = id / bands, band = id % bands;
  const int64_t i0 = seg * H, d0 = dstart + band * BW;
  auto none = [&]() {
    delta64[id] = 0.0f;
    if (delta32) delta32[id] = 0.0f;
  };
  if (d0 > N - 1 || i0 >= N - d0) {
    none();
    return;
  }
  auto range = [&](int64_t lo, int64_t hi, float& smax, float& smin, float& fmax_, float& gmax, float& mmax) {
    smax = 0.0f;
    smin = INFINITY;
    fmax_ = 0.0f;
    gmax = 0.0f;
    mmax = 0.0f;
    const int64_t b0 = lo / 64, b1 = (hi - 1) / 64 < nblk - 1 ? (hi - 1) / 64 : nblk - 1;
    for (int64_t b = b0; b <= b1; ++b) {
      smax = fmaxf(smax, bsw_max[b]);
      smin = fminf(smin, bsw_min[b]);
      fmax_ = fmaxf(fmax_, bdf_max[b]);
      gmax = fmaxf(gmax, bdg_max[b]);
      mmax = fmaxf(mmax, bmu_max[b]);
    }
  };
  float rsx, rsn, rfx, rgx, rmx, csx, csn, cfx, cgx, cmx;
  range(i0, i0 + H + 1, rsx, rsn, rfx, rgx, rmx);
  range(i0 + d0, i0 + d0 + H + BW + 1, csx, csn, cfx, cgx, cmx);
  if (!(rsn < INFINITY) || !(csn < INFINITY)) {
    none();  // no non-flat window on one side: nothing can pass
    return;
  }
  const double R = (double)H;
  const double phi = ((double)rsx / rsn) * ((double)csx / csn);
  const double psi = ((double)rfx * cgx + (double)rgx * cfx) / ((double)rsn * csn);
  const double xi = ((double)rfx + cfx) * (double)fmaxf(rmx, cmx) / ((double)rsn * csn);
  const double d64 = recurrence_bound(kEps64, R, phi, psi, xi, L);
  delta64[id] = d64 < 4.0 ? __double2float_ru(d64) : 4.0f;
  if (delta32) {
    const double d = recurrence_bound(kEps32, R, phi, psi, xi, L) + kFilter32;
    const float df_ = d < 1.0 ? __double2float_ru(d) : 1.0f;
    delta32[id] = df_;
    if (df_ > delta_max) hard[atomicAdd(nhard, 1ull)] = (int32_t)id;
  }
}

PassGrid pass_grid(int64_t N, int64_t e, int64_t dstart, int K, int64_t H) {
  PassGrid g;
  const int64_t ndiag = N - 1 - e;    // non-trivial diagonals e+1 .. N-1
  const int64_t nband = N - dstart;   // diagonals covered by the bands: dstart .. N-1
  const int64_t bw = (int64_t)kWave * K;
  g.bands = ndiag > 0 ? (nband + bw - 1) / bw : 0;
  g.segs = ndiag > 0 ? (N - dstart + H - 1) / H : 0;  // the first band has N - dstart rows
  g.cells = ndiag > 0 ? ndiag * (ndiag + 1) / 2 : 0;
  return g;
}

hipError_t launch_anchor(const double* xs, int64_t n, int L, bool init, int64_t H, int64_t dstart, int64_t segs,
                         int64_t stride, int64_t ncols, double* anc, hipStream_t st) {
  if (segs <= 0 || ncols <= 0) return hipSuccess;
  dim3 grid(blocks_for(ncols, 256), (unsigned)segs);
  if (init)
    k_anchor_init<<<grid, 256, 0, st>>>(xs, n, L, H, dstart, stride, ncols, anc);
  else
    k_anchor_grow<<<grid, 256, 0, st>>>(xs, n, L, H, dstart, stride, ncols, anc);
  return hipGetLastError();
}

// workgroups of a listed-items launch: two wavefronts per SIMD of the 256 CUs,
// as many as the FP64 collecting kernel keeps resident (229 VGPRs)
constexpr int64_t kListGrid = 2048;

template <typename T, int K>
static hipError_t launch_pass_k(const PassLaunch& p, hipStream_t st) {
  const PassGrid g = pass_grid(p.N, p.e, p.dstart, K, p.H);
  if (g.bands == 0) {  // nothing to launch: the timing events still mark an (empty) interval
    hipError_t e = p.ev_start ? hipEventRecord(p.ev_start, st) : hipSuccess;
    if (e == hipSuccess && p.ev_stop) e = hipEventRecord(p.ev_stop, st);
    return e;
  }
  PassArgs a;
  a.thr = p.thr;
  a.events = p.events;
  a.best = p.best;
  a.cnt = p.cnt;
  a.buf = p.buf;
  a.cap = p.cap;
  a.items = p.items;
  a.nitems = p.nitems_dev;
  a.delta = p.delta;
  a.delta_max = p.delta_max;
  a.N = p.N;
  a.e = p.e;
  a.H = p.H;
  a.dstart = p.dstart;
  a.anc_stride = p.anc_stride;
  a.anc_next = p.anc && p.grow ? const_cast<double*>(p.anc) : nullptr;
  a.bands = g.bands;
  a.L = p.L;
  if (p.items && (p.nitems <= 0 || !p.nitems_dev)) return p.nitems < 0 ? hipErrorInvalidValue : hipSuccess;
  const T* df = (const T*)(sizeof(T) == 8 ? (const void*)p.df : (const void*)p.df32);
  const T* dg = (const T*)(sizeof(T) == 8 ? (const void*)p.dg : (const void*)p.dg32);
  const T* inv = (const T*)(sizeof(T) == 8 ? (const void*)p.invn : (const void*)p.inv32);
  const T* thr = (const T*)(sizeof(T) == 8 ? (const void*)p.thr : (const void*)p.thr32);
  if (p.items) {
    // listed items (the FP64 re-run of FP32 items, collecting mode): a small
    // grid walks the list, so an empty or short list costs a few microseconds
    if constexpr (sizeof(T) == 8) {
      if (!p.append) return hipErrorInvalidValue;
      const dim3 grid((unsigned)(p.nitems < kListGrid ? p.nitems : kListGrid), 1);
      k_pass<T, K, MODE_APPEND, true><<<grid, kWave, 0, st>>>(df, dg, inv, thr, p.xs, p.anc, p.A, a);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  const dim3 grid((unsigned)g.segs, (unsigned)g.bands);
  if (p.ev_start || p.ev_stop) {
    if (p.append)
      hipExtLaunchKernelGGL(k_pass<T, K, MODE_APPEND, false>, grid, dim3(kWave), 0, st, p.ev_start, p.ev_stop, 0, df,
                            dg, inv, thr, p.xs, p.anc, p.A, a);
    else
      hipExtLaunchKernelGGL(k_pass<T, K, MODE_MP, false>, grid, dim3(kWave), 0, st, p.ev_start, p.ev_stop, 0, df, dg,
                            inv, thr, p.xs, p.anc, p.A, a);
  } else if (p.append) {
    k_pass<T, K, MODE_APPEND, false><<<grid, kWave, 0, st>>>(df, dg, inv, thr, p.xs, p.anc, p.A, a);
  } else {
    k_pass<T, K, MODE_MP, false><<<grid, kWave, 0, st>>>(df, dg, inv, thr, p.xs, p.anc, p.A, a);
  }
  return hipGetLastError();
}

hipError_t launch_pass(const PassLaunch& p, hipStream_t st) {
  if (p.fp32) {
    if (p.K == 8) return launch_pass_k<float, 8>(p, st);
    if (p.K == 4) return launch_pass_k<float, 4>(p, st);
    return hipErrorInvalidValue;
  }
  if (p.K == 8) return launch_pass_k<double, 8>(p, st);
  if (p.K == 4) return launch_pass_k<double, 4>(p, st);
  return hipErrorInvalidValue;
}

hipError_t launch_item_bounds(const float* bsw_max, const float* bsw_min, const float* bdf_max, const float* bdg_max,
                              const float* bmu_max, int64_t N, int64_t e, int64_t dstart, int K, int64_t H, int L,
                              float delta_max,
                              float* delta64, float* delta32, int32_t* hard, unsigned long long* nhard,
                              hipStream_t st) {
  const PassGrid g = pass_grid(N, e, dstart, K, H);
  const int64_t nitems = g.segs * g.bands;
  if (nitems == 0) return hipSuccess;
  if (!delta64 || (delta32 && (!hard || !nhard))) return hipErrorInvalidValue;
  const int64_t nblk = (N + 63) / 64;
  k_item_bounds<<<blocks_for(nitems, 256), 256, 0, st>>>(bsw_max, bsw_min, bdf_max, bdg_max, bmu_max, nblk, g.segs,
                                                         g.bands, H,
                                                         dstart, (int64_t)kWave * K, N, L, delta_max, delta64, delta32,
                                                         hard, nhard);
  return hipGetLastError();
}

}  // namespace valmod
