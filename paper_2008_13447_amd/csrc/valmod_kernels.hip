// HIP kernels of the VALMOD hot path for gfx950 (MI355X).
//
// Every kernel works on one series at one length L. Per-window arrays have
// N = n - L + 1 live entries followed by at least kPad zero entries, so column
// loads of the diagonal pass never need a bounds check.
#include "valmod_common.h"
#include "valmod_kernels.h"

#include <math.h>

namespace valmod {

// --------------------------------------------------------------------------
// Series conversion: input dtype -> FP64 working copy, zero padded; flags
// non-finite values.
template <typename TIn>
__global__ void k_convert(const TIn* __restrict__ in, int64_t n, int64_t npad, double* __restrict__ xs,
                          int* __restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  double v = i < n ? (double)in[i] : 0.0;
  if (i < n && !isfinite(v)) {
    atomicOr(err, 1);
    v = 0.0;
  }
  xs[i] = v;
}

// --------------------------------------------------------------------------
// Window statistics at length L (Eq. 6: mean and population deviation).
// Sums are anchored at the window's first value: A = sum(x - x0),
// B = sum((x - x0)^2). At the first length they are formed directly; each next
// length adds one term (the window grows by one point), so the cost is O(1) per
// window per length and no large-offset cancellation occurs.
__global__ void k_stats(const double* __restrict__ xs, int64_t N, int L, int first, double flat_eps,
                        double* __restrict__ A, double* __restrict__ B, double* __restrict__ mu,
                        double* __restrict__ sig, double* __restrict__ invn,
                        uint8_t* __restrict__ flat, unsigned long long* __restrict__ nflat) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool fl = false;
  if (i < N) {
    const double x0 = xs[i];
    double a, b;
    if (first) {
      a = 0.0;
      b = 0.0;
      for (int k = 1; k < L; ++k) {
        double d = xs[i + k] - x0;
        a += d;
        b = fma(d, d, b);
      }
    } else {
      a = A[i];
      b = B[i];
      double d = xs[i + L - 1] - x0;
      a += d;
      b = fma(d, d, b);
    }
    A[i] = a;
    B[i] = b;
    const double m = a / (double)L;
    double v = b / (double)L - m * m;
    v = v > 0.0 ? v : 0.0;
    const double s = sqrt(v);
    const double mval = x0 + m;
    fl = s <= flat_eps * fmax(1.0, fabs(mval));
    mu[i] = mval;
    sig[i] = s;
    flat[i] = fl ? 1 : 0;
    invn[i] = fl ? 0.0 : 1.0 / (s * sqrt((double)L));
  } else if (i < N + kPad) {
    mu[i] = 0.0;
    sig[i] = 0.0;
    flat[i] = 1;
    invn[i] = 0.0;
  }
  unsigned long long m = __ballot(fl);
  if ((threadIdx.x & (kWave - 1)) == 0 && m) atomicAdd(nflat, (unsigned long long)__popcll(m));
}

// --------------------------------------------------------------------------
// Co-moment recurrence inputs at length L. With C(i,j) = sum_k (x_{i+k} - mu_i)
// (x_{j+k} - mu_j), one diagonal step is
//   C(i+1, j+1) = C(i, j) + df_i * dg_j + df_j * dg_i,
//   df_i = (x_{i+L} - x_i) / 2,  dg_i = (x_{i+L} - mu_{i+1}) + (x_i - mu_i),
// which is the mean-centred form of the dot-product update of Alg.
// ComputeMatrixProfile (no cancellation at large offsets).
template <typename T>
__global__ void k_prep(const double* __restrict__ xs, const double* __restrict__ mu,
                       const double* __restrict__ sig, const double* __restrict__ invn, int64_t N, int L,
                       T* __restrict__ df, T* __restrict__ dg, float* __restrict__ sw32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N + kPad) return;
  double f = 0.0, g = 0.0;
  float w = INFINITY;
  if (i + 1 < N) {
    f = 0.5 * (xs[i + L] - xs[i]);
    g = (xs[i + L] - mu[i + 1]) + (xs[i] - mu[i]);
  }
  // sigma * sqrt(L), rounded down so that filter bounds built from it stay below the exact ones
  if (i < N && invn[i] > 0.0) w = __double2float_rd(sig[i] * sqrt((double)L));
  df[i] = (T)f;
  dg[i] = (T)g;
  sw32[i] = w;
}

// Centred FP64 correlation of windows o and c (both non-flat) at length L.
__device__ __forceinline__ double direct_rho(const double* __restrict__ xs, int L, int64_t o, int64_t c,
                                             double muo, double muc, double invo, double invc) {
  double acc = 0.0;
  for (int k = 0; k < L; ++k) acc = fma(xs[o + k] - muo, xs[c + k] - muc, acc);
  return acc * invo * invc;
}

// --------------------------------------------------------------------------
// Seeds of the MP-mode thresholds: for each owner a few real candidates whose
// exact correlation gives a starting best key (any real candidate is a valid
// starting point for a running minimum). Candidates: the owner's neighbour at
// the previous length and its neighbours' neighbours shifted along the
// diagonal, plus the nearest non-trivial windows.
__global__ void k_seed_mp(const double* __restrict__ xs, const double* __restrict__ mu,
                          const double* __restrict__ invn, const uint8_t* __restrict__ flat,
                          const int32_t* __restrict__ prev_idx, int64_t N, int L, int64_t e,
                          uint64_t* __restrict__ best, double* __restrict__ thr, float* __restrict__ thr32) {
  int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N + kPad) return;
  if (o >= N || flat[o]) {
    best[o] = kEmptyKey;
    thr[o] = 3.0;  // padding and flat owners accept nothing
    thr32[o] = 3.0f;
    return;
  }
  int64_t cand[5];
  int nc = 0;
  if (prev_idx) {
    int64_t c0 = prev_idx[o];
    if (c0 >= 0) cand[nc++] = c0;
    if (o > 0 && prev_idx[o - 1] >= 0) cand[nc++] = prev_idx[o - 1] + 1;
    if (o + 1 < N && prev_idx[o + 1] >= 0) cand[nc++] = prev_idx[o + 1] - 1;
  }
  cand[nc++] = o + e + 1;
  cand[nc++] = o - e - 1;
  uint64_t kbest = kEmptyKey;
  const double muo = mu[o], invo = invn[o];
  for (int s = 0; s < nc; ++s) {
    int64_t c = cand[s];
    if (c < 0 || c >= N || iabs64(c - o) <= e || flat[c]) continue;
    double r = direct_rho(xs, L, o, c, muo, mu[c], invo, invn[c]);
    uint64_t k = make_key(r, c);
    kbest = k < kbest ? k : kbest;
  }
  best[o] = kbest;
  const double th = key_threshold(kbest);
  thr[o] = th;
  thr32[o] = __double2float_rd(th);
}

// --------------------------------------------------------------------------
// Anchor table of the diagonal pass (the first-row dot products of
// Alg. ComputeMatrixProfile, one per work item and diagonal):
//   S(i0, i0 + d) = sum_{k<L} (x_{i0+k} - x_{i0}) (x_{i0+d+k} - x_{i0+d})
// for every segment start row i0 = seg * H and diagonal d >= dstart. Values
// are excursions from each window's first point (no large-offset
// cancellation); the pass turns them into co-moments with C = S - A_i A_j / L.
// k_anchor_init forms them directly (L FMAs each); when the length grows by one
// k_anchor_grow adds the single new term, so later lengths cost O(1) per anchor.
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
// The per-cell work is two FMAs and one compare. The compare is a filter in
// co-moment space: for owner thresholds thr (in correlation units) the cell can
// matter only if rho = C / (sw_i sw_j) >= min(thr_i, thr_j), with
// sw = sigma * sqrt(L). Over a block of K rows the filter uses
//   tau_j = min(thr_j, min_rows thr_i) * sw_j * min_rows sw_i   (times 1 - 1e-12),
// which is never larger than the exact per-cell bound, so no qualifying cell is
// skipped. Cells that pass go to a slow path that evaluates rho exactly and
// applies the mode's action:
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
  double* thr;         // per-owner threshold (correlation units)
  uint64_t* best;      // MODE_MP: packed best key per owner
  uint32_t* cnt;       // MODE_APPEND: candidates appended per owner
  int32_t* buf;        // MODE_APPEND: owner-major candidate lists
  int64_t cap;         // MODE_APPEND: list capacity per owner
  unsigned long long* events;  // [0] wave-steps that took the slow path, [1] owner hits
  int64_t anc_stride;  // anchor-table row length (diagonals per segment row)
  int64_t N, e, H, dstart;
  int L;
};

template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t off) {
  return *(const T*)((const char*)base + off);
}

// Wide per-lane loads of `n` consecutive doubles (lanes read adjacent ranges,
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

// Per-wavefront LDS queue of slow-path results. The step loop issues no global
// writes or atomics (on gfx9 they share the load counter with the prefetch
// loads, and a write inside a data-dependent branch makes every later wait
// drain all prefetches); the queue is flushed to global memory when it could
// overflow at the next step and at the end of the work item.
constexpr int kQueue = 1024;

// min of two thresholds (never NaN) without the IEEE quieting of the operands
// that fmin() implies.
__device__ __forceinline__ double vmin_f64(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

template <int K, int MODE>
__global__ __launch_bounds__(kWave) void k_pass(const double* __restrict__ g_df, const double* __restrict__ g_dg,
                                                const double* __restrict__ g_invn, const double* __restrict__ g_thr,
                                                const double* __restrict__ g_anc, const double* __restrict__ g_A,
                                                PassArgs a) {
  // g_thr aliases a.thr: threshold reads through it may return values older than
  // this kernel's own updates, which only makes the filter looser (never unsound).
  static_assert(K % 4 == 0, "K must be a multiple of 4");
  constexpr int64_t BW = (int64_t)kWave * K;  // diagonals per band
  constexpr int HK = K / 2;
  __shared__ int32_t q_owner[kQueue];
  __shared__ uint64_t q_val[kQueue];  // MODE_MP: packed key; MODE_APPEND: candidate index
  const int t = threadIdx.x;
  const int64_t N = a.N;
  const int64_t d0 = a.dstart + (int64_t)blockIdx.y * BW;
  if (d0 > N - 1) return;
  const int64_t i0 = (int64_t)blockIdx.x * a.H;
  const int64_t rowEnd = N - d0;
  if (i0 >= rowEnd) return;
  const int rows = (int)((i0 + a.H < rowEnd ? i0 + a.H : rowEnd) - i0);
  const int64_t dl = d0 + (int64_t)K * t;

  // co-moments at row i0 from the FP64 anchor table: C = S - A_i A_j / L
  double C[K];
  {
    double S[K], Aj[K];
    load_run<K>(g_anc + (int64_t)blockIdx.x * a.anc_stride + (dl - a.dstart), S);
    load_run<K>(g_A + i0 + dl, Aj);
    const double Ai = g_A[i0] / (double)a.L;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int64_t j = i0 + dl + q;
      C[q] = (dl + q > a.e && j < N) ? S[q] - Ai * Aj[q] : -INFINITY;  // trivial or past the end
    }
  }

  // Column window: at step u of a block, slot s holds column i + dl + ((s - u) mod K).
  // Two register sets X and Y alternate by block: during a block whose slots
  // start in set P, slot s moves to set Q (holding the column that enters) at
  // step s, and the freed entries of P receive the next block's entering
  // columns, a half block at a time. No register copies are needed.
  double Xdf[K], Xdg[K], Xinv[K], Xthr[K];
  double Ydf[K], Ydg[K], Yinv[K], Ythr[K];
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

  auto flush = [&]() {
    __syncthreads();
    for (int b = 0; b < qn; b += kWave) {
      if (b + t < qn) {
        const int32_t own = q_owner[b + t];
        const uint64_t v = q_val[b + t];
        if (MODE == MODE_MP) {
          atomicMin((unsigned long long*)&a.best[own], (unsigned long long)v);
          const double nt = key_threshold(v);
          if (nt > a.thr[own]) a.thr[own] = nt;  // racy but every stored value is a real candidate's bound
        } else {
          const uint32_t pos = atomicAdd(&a.cnt[own], 1u);
          if ((int64_t)pos < a.cap) a.buf[(int64_t)own * a.cap + pos] = (int32_t)v;
        }
      }
    }
    if (a.events && t == 0) atomicAdd(&a.events[1], (unsigned long long)qn);
    __syncthreads();
    qn = 0;
  };
  auto push = [&](bool want, int32_t owner, uint64_t val) {
    const uint64_t m = __ballot(want);
    if (!m) return;
    if (want) {
      const int pos = qn + __popcll(m & ((uint64_t(1) << t) - 1));
      q_owner[pos] = owner;
      q_val[pos] = val;
    }
    qn += __popcll(m);
  };

  // one block of K rows starting at row ib; slots start in P and move to Q
  auto block = [&](int64_t ib, double* Pdf, double* Pdg, double* Pinv, double* Pthr, double* Qdf, double* Qdg,
                   double* Qinv, double* Qthr) {
    double rdf[K], rdg[K], rinv[K], rthr[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      rdf[u] = g_df[ib + u];
      rdg[u] = g_dg[ib + u];
      rinv[u] = g_invn[ib + u];
      rthr[u] = g_thr[ib + u];
    }
    const int64_t cn = ib + dl + 2 * K;  // first column entering during the next block
    // Every block runs all K steps: rows past the segment or the series only meet
    // columns past the end (zero inverse norm, padded thresholds), so they never
    // produce a queue entry, and all their reads stay inside the zero padding.
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int64_t i = ib + u;
      // exact correlation of every cell and the test against both owners' thresholds
      bool pass = false;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int s = (q + u) % K;
        const double inv = s < u ? Qinv[s] : Pinv[s];
        const double th = s < u ? Qthr[s] : Pthr[s];
        pass |= (C[q] * inv) * rinv[u] >= vmin_f64(th, rthr[u]);
      }
      if (__any(pass)) {
        ++ev_steps;
        if (qn + kWave * K + 1 > kQueue) flush();
        uint64_t rowkey = kEmptyKey;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const int s = (q + u) % K;
          const int64_t j = i + dl + q;
          const double inv = s < u ? Qinv[s] : Pinv[s];
          double& th = s < u ? Qthr[s] : Pthr[s];
          const double rho = (C[q] * inv) * rinv[u];
          const bool ok = j < N && rinv[u] > 0.0 && inv > 0.0;
          const bool col = ok && rho >= th;
          if (MODE == MODE_MP) {
            const uint64_t key = col ? make_key(rho, i) : kEmptyKey;
            push(col, (int32_t)j, key);
            if (col) {
              const double nt = key_threshold(key);
              th = nt > th ? nt : th;
            }
            if (ok && rho >= rthr[u]) {
              const uint64_t k2 = make_key(rho, j);
              rowkey = k2 < rowkey ? k2 : rowkey;
            }
          } else {
            push(col, (int32_t)j, (uint64_t)i);
            push(ok && rho >= rthr[u], (int32_t)i, (uint64_t)j);
          }
        }
        if (MODE == MODE_MP && __any(rowkey != kEmptyKey)) {
          rowkey = wave_min_u64(rowkey);
          push(t == 0, (int32_t)i, rowkey);
        }
      }
      // advance every diagonal one row: C(i+1, j+1) = C(i, j) + df_i dg_j + df_j dg_i
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int s = (q + u) % K;
        const double cdf = s < u ? Qdf[s] : Pdf[s];
        const double cdg = s < u ? Qdg[s] : Pdg[s];
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
}

// --------------------------------------------------------------------------
// Matrix-profile entries at L from the best keys: the FP64 distance of every
// chosen pair is evaluated directly from the z-normalised windows (no closed
// form, exact near d = 0), in a canonical (min, max) order so d(i, j) = d(j, i)
// bit for bit. Also applies Alg. updateVALMP (strictly smaller normalised
// distance wins, so the shorter length keeps ties).
__global__ void k_finalize(const double* __restrict__ xs, const double* __restrict__ mu,
                           const double* __restrict__ sig, const uint64_t* __restrict__ best,
                           int64_t N, int L, double* __restrict__ prof_dist,
                           int32_t* __restrict__ prof_idx, double* __restrict__ valmp_norm,
                           double* __restrict__ valmp_dist, int32_t* __restrict__ valmp_len,
                           int32_t* __restrict__ valmp_idx) {
  int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  const uint64_t key = best[o];
  double d = INFINITY;
  int32_t c32 = -1;
  if (key != kEmptyKey) {
    const int64_t c = key_cand(key);
    const int64_t a = o < c ? o : c, b = o < c ? c : o;
    const double ma = mu[a], mb = mu[b];
    const double ia = 1.0 / sig[a], ib = 1.0 / sig[b];
    double acc = 0.0;
    for (int k = 0; k < L; ++k) {
      const double z = (xs[a + k] - ma) * ia - (xs[b + k] - mb) * ib;
      acc = fma(z, z, acc);
    }
    d = sqrt(acc);
    c32 = (int32_t)c;
  }
  if (prof_dist) prof_dist[o] = d;
  if (prof_idx) prof_idx[o] = c32;
  if (valmp_norm) {
    const double nd = d * sqrt(1.0 / (double)L);
    if (nd < valmp_norm[o]) {
      valmp_norm[o] = nd;
      if (valmp_dist) valmp_dist[o] = d;
      if (valmp_len) valmp_len[o] = L;
      if (valmp_idx) valmp_idx[o] = c32;
    }
  }
}

// Per-length diagnostic counters: copies the running device counters into the
// stats row of length t and clears them.
__global__ void k_record_stats(unsigned long long* __restrict__ cnt, int64_t* __restrict__ row, int full_pass,
                               int64_t valid, int64_t failed, int64_t recomputed) {
  if (threadIdx.x != 0) return;
  if (row) {
    row[0] = valid;
    row[1] = failed;
    row[2] = recomputed;
    row[3] = full_pass;
    row[4] = (int64_t)cnt[1];
    row[5] = (int64_t)cnt[4];
    row[6] = (int64_t)cnt[2];
    row[7] = (int64_t)cnt[3];
  }
  cnt[1] = cnt[2] = cnt[3] = cnt[4] = 0;
}

__global__ void k_fill_tail(int64_t from, int64_t to, double* __restrict__ prof_dist,
                            int32_t* __restrict__ prof_idx) {
  int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= to) return;
  if (prof_dist) prof_dist[i] = INFINITY;
  if (prof_idx) prof_idx[i] = -1;
}

__global__ void k_valmp_init(int64_t N0, double* __restrict__ norm, double* __restrict__ dist,
                             int32_t* __restrict__ len, int32_t* __restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N0) return;
  norm[i] = INFINITY;
  if (dist) dist[i] = INFINITY;
  if (len) len[i] = 0;
  if (idx) idx[i] = -1;
}

// --------------------------------------------------------------------------
// Rankings. One workgroup per length; k greedy rounds, each a block-wide
// lexicographic arg-min over the profile that skips candidates within the
// exclusion zone of an already accepted endpoint.
constexpr int kRankThreads = 1024;
constexpr int kMaxK = 64;

struct MotifKey {
  double d;
  int32_t a, b;
};

__device__ __forceinline__ bool motif_less(const MotifKey& u, const MotifKey& v) {
  if (u.d != v.d) return u.d < v.d;
  if (u.a != v.a) return u.a < v.a;
  return u.b < v.b;
}

template <typename Key, typename Less>
__device__ Key block_reduce(Key v, Less less, Key* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s && less(sh[t + s], sh[t])) sh[t] = sh[t + s];
    __syncthreads();
  }
  Key r = sh[0];
  __syncthreads();
  return r;
}

// Per length t: motif pairs (C14 reading: sort by (d, min, max), greedy with
// the exclusion zone on all four endpoint combinations).
__global__ __launch_bounds__(kRankThreads) void k_topk_motifs(
    const double* __restrict__ prof_dist, const int32_t* __restrict__ prof_idx, int64_t N0,
    int64_t n, int l_min, int excl_den, int k, int32_t* __restrict__ motif_ab, double* __restrict__ motif_d) {
  __shared__ MotifKey sh[kRankThreads];
  __shared__ int32_t acc_a[kMaxK], acc_b[kMaxK];
  const int tl = blockIdx.x;
  const int L = l_min + tl;
  const int64_t N = n - L + 1;
  const int64_t e = excl_zone(L, excl_den);
  const double* dist = prof_dist + (int64_t)tl * N0;
  const int32_t* idx = prof_idx + (int64_t)tl * N0;
  int got = 0;
  for (int r = 0; r < k; ++r) {
    MotifKey best{INFINITY, 0x7fffffff, 0x7fffffff};
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
      const int32_t c = idx[i];
      const double d = dist[i];
      if (c < 0 || !(d < INFINITY)) continue;
      MotifKey m{d, (int32_t)(i < c ? i : c), (int32_t)(i < c ? c : i)};
      if (!motif_less(m, best)) continue;
      bool ok = true;
      for (int s = 0; s < got; ++s) {
        if (iabs64(m.a - acc_a[s]) <= e || iabs64(m.a - acc_b[s]) <= e ||
            iabs64(m.b - acc_a[s]) <= e || iabs64(m.b - acc_b[s]) <= e) {
          ok = false;
          break;
        }
      }
      if (ok) best = m;
    }
    best = block_reduce(best, motif_less, sh);
    if (!(best.d < INFINITY)) break;
    if (threadIdx.x == 0) {
      acc_a[got] = best.a;
      acc_b[got] = best.b;
      motif_ab[((int64_t)tl * k + got) * 2] = best.a;
      motif_ab[((int64_t)tl * k + got) * 2 + 1] = best.b;
      motif_d[(int64_t)tl * k + got] = best.d;
    }
    __syncthreads();
    ++got;
  }
  for (int r = got + threadIdx.x; r < k; r += blockDim.x) {
    motif_ab[((int64_t)tl * k + r) * 2] = -1;
    motif_ab[((int64_t)tl * k + r) * 2 + 1] = -1;
    motif_d[(int64_t)tl * k + r] = NAN;
  }
}

struct DiscordKey {
  double d;
  int32_t i, nn;
};

__device__ __forceinline__ bool discord_less(const DiscordKey& u, const DiscordKey& v) {
  // "less" = better: larger distance first, then smaller offset
  if (u.d != v.d) return u.d > v.d;
  return u.i < v.i;
}

// Per length t: top-k 1st discords (C15 reading: descending MP over finite
// entries, ties to the smaller offset, exclusion zone around accepted offsets).
__global__ __launch_bounds__(kRankThreads) void k_topk_discords(
    const double* __restrict__ prof_dist, const int32_t* __restrict__ prof_idx, int64_t N0,
    int64_t n, int l_min, int excl_den, int k, int32_t* __restrict__ discord_on,
    double* __restrict__ discord_d) {
  __shared__ DiscordKey sh[kRankThreads];
  __shared__ int32_t acc_i[kMaxK];
  const int tl = blockIdx.x;
  const int L = l_min + tl;
  const int64_t N = n - L + 1;
  const int64_t e = excl_zone(L, excl_den);
  const double* dist = prof_dist + (int64_t)tl * N0;
  const int32_t* idx = prof_idx + (int64_t)tl * N0;
  int got = 0;
  for (int r = 0; r < k; ++r) {
    DiscordKey best{-INFINITY, 0x7fffffff, -1};
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
      const int32_t c = idx[i];
      const double d = dist[i];
      if (c < 0 || !(d < INFINITY)) continue;
      DiscordKey m{d, (int32_t)i, c};
      if (!discord_less(m, best)) continue;
      bool ok = true;
      for (int s = 0; s < got; ++s)
        if (iabs64((int64_t)i - acc_i[s]) <= e) {
          ok = false;
          break;
        }
      if (ok) best = m;
    }
    best = block_reduce(best, discord_less, sh);
    if (best.nn < 0) break;
    if (threadIdx.x == 0) {
      acc_i[got] = best.i;
      discord_on[((int64_t)tl * k + got) * 2] = best.i;
      discord_on[((int64_t)tl * k + got) * 2 + 1] = best.nn;
      discord_d[(int64_t)tl * k + got] = best.d;
    }
    __syncthreads();
    ++got;
  }
  for (int r = got + threadIdx.x; r < k; r += blockDim.x) {
    discord_on[((int64_t)tl * k + r) * 2] = -1;
    discord_on[((int64_t)tl * k + r) * 2 + 1] = -1;
    discord_d[(int64_t)tl * k + r] = NAN;
  }
}

struct GMotifKey {
  double dn;
  int32_t L, i;
};

__device__ __forceinline__ bool gmotif_less(const GMotifKey& u, const GMotifKey& v) {
  if (u.dn != v.dn) return u.dn < v.dn;
  if (u.L != v.L) return u.L < v.L;
  return u.i < v.i;
}

// Cross-length rankings of one series. Discords: for each rank, the
// position-wise max over lengths of d / sqrt(L), strictly (shorter length wins
// ties; Alg. UpdateVariableLengthDiscords). Motifs: VALMP entries by
// (normalised d, length, offset), greedy with the exclusion zone of the longer
// of the two lengths.
__global__ __launch_bounds__(kRankThreads) void k_global_rank(
    const double* __restrict__ valmp_norm, const double* __restrict__ valmp_dist,
    const int32_t* __restrict__ valmp_len, const int32_t* __restrict__ valmp_idx, int64_t N0,
    const int32_t* __restrict__ discord_on, const double* __restrict__ discord_d, int nlen, int l_min,
    int excl_den, int km, int kd, int32_t* __restrict__ g_motif_abl, double* __restrict__ g_motif_d,
    int32_t* __restrict__ g_discord_onl, double* __restrict__ g_discord_d) {
  __shared__ GMotifKey sh[kRankThreads];
  __shared__ int32_t acc_a[kMaxK], acc_b[kMaxK], acc_L[kMaxK];
  if (g_discord_onl && discord_d) {
    for (int r = threadIdx.x; r < kd; r += blockDim.x) {
      double bestdn = -INFINITY;
      int32_t o = -1, nn = -1, Lb = -1;
      double db = NAN, dnb = NAN;
      for (int t = 0; t < nlen; ++t) {
        const double d = discord_d[(int64_t)t * kd + r];
        if (!(d == d)) continue;
        const int L = l_min + t;
        const double dn = d / sqrt((double)L);
        if (dn > bestdn) {
          bestdn = dn;
          o = discord_on[((int64_t)t * kd + r) * 2];
          nn = discord_on[((int64_t)t * kd + r) * 2 + 1];
          Lb = L;
          db = d;
          dnb = dn;
        }
      }
      g_discord_onl[r * 3] = o;
      g_discord_onl[r * 3 + 1] = nn;
      g_discord_onl[r * 3 + 2] = Lb;
      g_discord_d[r * 2] = db;
      g_discord_d[r * 2 + 1] = dnb;
    }
  }
  if (!g_motif_abl) return;
  int got = 0;
  for (int r = 0; r < km; ++r) {
    GMotifKey best{INFINITY, 0x7fffffff, 0x7fffffff};
    for (int64_t i = threadIdx.x; i < N0; i += blockDim.x) {
      const int32_t c = valmp_idx[i];
      const double dn = valmp_norm[i];
      if (c < 0 || !(dn < INFINITY)) continue;
      GMotifKey m{dn, valmp_len[i], (int32_t)i};
      if (!gmotif_less(m, best)) continue;
      const int64_t a = i < c ? i : c, b = i < c ? c : i;
      bool ok = true;
      for (int s = 0; s < got; ++s) {
        const int64_t Lm = m.L > acc_L[s] ? m.L : acc_L[s];
        const int64_t e = excl_zone(Lm, excl_den);
        if (iabs64(a - acc_a[s]) <= e || iabs64(a - acc_b[s]) <= e || iabs64(b - acc_a[s]) <= e ||
            iabs64(b - acc_b[s]) <= e) {
          ok = false;
          break;
        }
      }
      if (ok) best = m;
    }
    best = block_reduce(best, gmotif_less, sh);
    if (!(best.dn < INFINITY)) break;
    if (threadIdx.x == 0) {
      const int32_t i = best.i, c = valmp_idx[i];
      acc_a[got] = i < c ? i : c;
      acc_b[got] = i < c ? c : i;
      acc_L[got] = best.L;
      g_motif_abl[got * 3] = acc_a[got];
      g_motif_abl[got * 3 + 1] = acc_b[got];
      g_motif_abl[got * 3 + 2] = best.L;
      g_motif_d[got * 2] = valmp_dist[i];
      g_motif_d[got * 2 + 1] = best.dn;
    }
    __syncthreads();
    ++got;
  }
  for (int r = got + threadIdx.x; r < km; r += blockDim.x) {
    g_motif_abl[r * 3] = g_motif_abl[r * 3 + 1] = g_motif_abl[r * 3 + 2] = -1;
    g_motif_d[r * 2] = g_motif_d[r * 2 + 1] = NAN;
  }
}

// --------------------------------------------------------------------------
// Host-side launch wrappers (no allocation, no synchronisation).

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

hipError_t launch_convert(const void* in, int dtype, int64_t n, int64_t npad, double* xs, int* err,
                          hipStream_t st) {
  if (dtype == 0)
    k_convert<float><<<blocks_for(npad, 256), 256, 0, st>>>((const float*)in, n, npad, xs, err);
  else
    k_convert<double><<<blocks_for(npad, 256), 256, 0, st>>>((const double*)in, n, npad, xs, err);
  return hipGetLastError();
}

hipError_t launch_stats(const double* xs, int64_t N, int L, int first, double flat_eps, double* A,
                        double* B, double* mu, double* sig, double* invn, uint8_t* flat,
                        unsigned long long* nflat, hipStream_t st) {
  k_stats<<<blocks_for(N + kPad, 256), 256, 0, st>>>(xs, N, L, first, flat_eps, A, B, mu, sig, invn,
                                                       flat, nflat);
  return hipGetLastError();
}

hipError_t launch_prep_f64(const double* xs, const double* mu, const double* sig, const double* invn, int64_t N,
                           int L, double* df, double* dg, float* sw32, hipStream_t st) {
  k_prep<double><<<blocks_for(N + kPad, 256), 256, 0, st>>>(xs, mu, sig, invn, N, L, df, dg, sw32);
  return hipGetLastError();
}

hipError_t launch_seed_mp(const double* xs, const double* mu, const double* invn, const uint8_t* flat,
                          const int32_t* prev_idx, int64_t N, int L, int64_t e, uint64_t* best,
                          double* thr, float* thr32, hipStream_t st) {
  k_seed_mp<<<blocks_for(N + kPad, 128), 128, 0, st>>>(xs, mu, invn, flat, prev_idx, N, L, e, best, thr, thr32);
  return hipGetLastError();
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

template <int K>
static hipError_t launch_pass_k(const PassLaunch& p, hipStream_t st) {
  const PassGrid g = pass_grid(p.N, p.e, p.dstart, K, p.H);
  if (g.bands == 0) return hipSuccess;
  PassArgs a;
  a.thr = p.thr;
  a.events = p.events;
  a.best = p.best;
  a.cnt = p.cnt;
  a.buf = p.buf;
  a.cap = p.cap;
  a.N = p.N;
  a.e = p.e;
  a.H = p.H;
  a.dstart = p.dstart;
  a.anc_stride = p.anc_stride;
  a.L = p.L;
  dim3 grid((unsigned)g.segs, (unsigned)g.bands);
  if (p.append)
    k_pass<K, MODE_APPEND><<<grid, kWave, 0, st>>>(p.df, p.dg, p.invn, p.thr, p.anc, p.A, a);
  else
    k_pass<K, MODE_MP><<<grid, kWave, 0, st>>>(p.df, p.dg, p.invn, p.thr, p.anc, p.A, a);
  return hipGetLastError();
}

hipError_t launch_pass(const PassLaunch& p, hipStream_t st) {
  if (p.K == 8) return launch_pass_k<8>(p, st);
  if (p.K == 4) return launch_pass_k<4>(p, st);
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const double* xs, const double* mu, const double* sig, const uint64_t* best,
                           int64_t N, int L, double* prof_dist, int32_t* prof_idx, double* valmp_norm,
                           double* valmp_dist, int32_t* valmp_len, int32_t* valmp_idx, hipStream_t st) {
  k_finalize<<<blocks_for(N, 128), 128, 0, st>>>(xs, mu, sig, best, N, L, prof_dist, prof_idx, valmp_norm,
                                                 valmp_dist, valmp_len, valmp_idx);
  return hipGetLastError();
}

hipError_t launch_record_stats(unsigned long long* cnt, int64_t* row, int full_pass, int64_t valid,
                               int64_t failed, int64_t recomputed, hipStream_t st) {
  k_record_stats<<<1, 64, 0, st>>>(cnt, row, full_pass, valid, failed, recomputed);
  return hipGetLastError();
}

hipError_t launch_fill_tail(int64_t from, int64_t to, double* prof_dist, int32_t* prof_idx, hipStream_t st) {
  if (to <= from) return hipSuccess;
  k_fill_tail<<<blocks_for(to - from, 256), 256, 0, st>>>(from, to, prof_dist, prof_idx);
  return hipGetLastError();
}

hipError_t launch_valmp_init(int64_t N0, double* norm, double* dist, int32_t* len, int32_t* idx,
                             hipStream_t st) {
  k_valmp_init<<<blocks_for(N0, 256), 256, 0, st>>>(N0, norm, dist, len, idx);
  return hipGetLastError();
}

hipError_t launch_rankings(const double* prof_dist, const int32_t* prof_idx, int64_t N0, int64_t n, int l_min,
                           int nlen, int excl_den, int km, int kd, int32_t* motif_ab, double* motif_d,
                           int32_t* discord_on, double* discord_d, hipStream_t st) {
  if (motif_ab && motif_d)
    k_topk_motifs<<<nlen, kRankThreads, 0, st>>>(prof_dist, prof_idx, N0, n, l_min, excl_den, km, motif_ab,
                                                 motif_d);
  if (discord_on && discord_d)
    k_topk_discords<<<nlen, kRankThreads, 0, st>>>(prof_dist, prof_idx, N0, n, l_min, excl_den, kd, discord_on,
                                                   discord_d);
  return hipGetLastError();
}

hipError_t launch_global_rank(const double* valmp_norm, const double* valmp_dist, const int32_t* valmp_len,
                              const int32_t* valmp_idx, int64_t N0, const int32_t* discord_on,
                              const double* discord_d, int nlen, int l_min, int excl_den, int km, int kd,
                              int32_t* g_motif_abl, double* g_motif_d, int32_t* g_discord_onl,
                              double* g_discord_d, hipStream_t st) {
  k_global_rank<<<1, kRankThreads, 0, st>>>(valmp_norm, valmp_dist, valmp_len, valmp_idx, N0, discord_on,
                                            discord_d, nlen, l_min, excl_den, km, kd, g_motif_abl, g_motif_d,
                                            g_discord_onl, g_discord_d);
  return hipGetLastError();
}

}  // namespace valmod
