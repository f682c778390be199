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
// Per-window inputs at length L, in one pass over the windows.
//
// Statistics (Eq. 6: mean and population deviation). Sums are anchored at the
// window's first value: A = sum(x - x0), B = sum((x - x0)^2). At the first
// length they are formed directly; each next length adds one term (the window
// grows by one point) to the previous length's sums (A_in, B_in -> A_out,
// B_out: two buffers, so no window reads a neighbour's updated sum), so the
// cost is O(1) per window per length and no large-offset cancellation occurs.
//
// Co-moment recurrence inputs. With C(i,j) = sum_k (x_{i+k} - mu_i)(x_{j+k} - mu_j),
// one diagonal step is
//   C(i+1, j+1) = C(i, j) + df_i * dg_j + df_j * dg_i,
//   df_i = (x_{i+L} - x_i) / 2,  dg_i = (x_{i+L} - mu_{i+1}) + (x_i - mu_i),
// which is the mean-centred form of the dot-product update of Alg.
// ComputeMatrixProfile (no cancellation at large offsets). mu_{i+1} comes from
// the next lane; the last lane of a wavefront forms it itself.
//
// F32: also the FP32 copies of df, dg and the inverse norms for the FP32 pass
// (nearest rounding: their error is part of the item bound; a flat or padded
// window, whose inverse norm is zero, gets NaN so that every correlation it
// enters fails every threshold test). Per block of 64 windows, the extrema of
// sigma sqrt(L), |df| and |dg| that bound the rounding of the recurrence in
// either precision, rounded outward.
//
// With partial profiles at base b (hflat non-null): the largest ratio
// sigma_b / sigma_L over the windows that were flat at b (never stored in a
// partial profile) but are candidates at L goes to *rflat (bits of a
// non-negative double): such a window c is at distance at least
// sqrt(b) (sigma_{o,b} / sigma_{o,L} - sigma_{c,b} / sigma_{c,L}) from any owner o
// (the base-length part of the distance, minimised over the offset, with the
// correlation at b at most 1), which the sweep folds into its bound.
template <bool F32>
__global__ __launch_bounds__(256) void k_window_prep(
    const double* __restrict__ xs, int64_t N, int L, int first, double flat_eps, const double* __restrict__ A_in,
    const double* __restrict__ B_in, double* __restrict__ A_out, double* __restrict__ B_out, double* __restrict__ mu,
    double* __restrict__ sig, double* __restrict__ invn, uint8_t* __restrict__ flat,
    unsigned long long* __restrict__ nflat, double* __restrict__ df, double* __restrict__ dg,
    float* __restrict__ sw32, float* __restrict__ df32, float* __restrict__ dg32, float* __restrict__ inv32,
    float* __restrict__ bsw_max, float* __restrict__ bsw_min, float* __restrict__ bdf_max,
    float* __restrict__ bdg_max, float* __restrict__ bmu_max, const uint8_t* __restrict__ hflat,
    const double* __restrict__ hsig, unsigned long long* __restrict__ rflat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  // anchored sums of window w at this length
  auto sums = [&](int64_t w, double& a, double& b) {
    const double x0 = xs[w];
    if (first) {
      a = 0.0;
      b = 0.0;
      for (int k = 1; k < L; ++k) {
        const double d = xs[w + k] - x0;
        a += d;
        b = fma(d, d, b);
      }
    } else {
      a = A_in[w];
      b = B_in[w];
      const double d = xs[w + L - 1] - x0;
      a += d;
      b = fma(d, d, b);
    }
  };
  const bool live = i < N;
  bool fl = false;
  double mval = 0.0, s = 0.0, inv = 0.0;
  if (live) {
    double a, b;
    sums(i, a, b);
    A_out[i] = a;
    B_out[i] = b;
    const double m = a / (double)L;
    double v = b / (double)L - m * m;
    v = v > 0.0 ? v : 0.0;
    s = sqrt(v);
    mval = xs[i] + m;
    fl = s <= flat_eps * fmax(1.0, fabs(mval));
    inv = fl ? 0.0 : 1.0 / (s * sqrt((double)L));
  }
  // the next window's mean (same arithmetic as its own lane)
  double mnext = __shfl_down(mval, 1, kWave);
  if (lane == kWave - 1 && i + 1 < N) {
    double a, b;
    sums(i + 1, a, b);
    mnext = xs[i + 1] + a / (double)L;
  }
  const unsigned long long fm = __ballot(fl);
  if (lane == 0 && fm) atomicAdd(nflat, (unsigned long long)__popcll(fm));
  if (hflat) {
    double r = 0.0;  // non-negative: its bit pattern orders like its value
    if (live && !fl && hflat[i]) r = hsig[i] / s;
    r = wave_max_f64(r);
    if (lane == 0 && r > 0.0) atomicMax(rflat, (unsigned long long)__double_as_longlong(r));
  }
  if (i >= N + kPad) return;
  mu[i] = live ? mval : 0.0;
  sig[i] = live ? s : 0.0;
  flat[i] = live ? (fl ? 1 : 0) : 1;
  invn[i] = inv;
  double f = 0.0, g = 0.0;
  if (i + 1 < N) {
    f = 0.5 * (xs[i + L] - xs[i]);
    g = (xs[i + L] - mnext) + (xs[i] - mval);
  }
  df[i] = f;
  dg[i] = g;
  // sigma * sqrt(L), rounded down so that filter bounds built from it stay below the exact ones
  sw32[i] = (live && inv > 0.0) ? __double2float_rd(s * sqrt((double)L)) : INFINITY;
  if (F32) {
    df32[i] = (float)f;
    dg32[i] = (float)g;
    inv32[i] = inv > 0.0 ? (float)inv : __int_as_float(0x7fc00000);
  }
  if (bsw_max) {
    // blocks of 64 windows are whole wavefronts (blockDim is a multiple of 64)
    const int64_t blk = i / kWave;
    if (blk * kWave < N) {
      double smax = 0.0, smin = INFINITY, fmx = 0.0, gmx = 0.0, mmx = 0.0;
      if (live) {
        if (inv > 0.0) {
          const double w = s * sqrt((double)L);
          smax = w;
          smin = w;
        }
        fmx = fabs(f);
        gmx = fabs(g);
        mmx = fabs(mval);
        if (lane == kWave - 1 && i + 1 < N) mmx = fmax(mmx, fabs(mnext));  // dg reads the next mean too
      }
      smax = wave_max_f64(smax);
      smin = wave_min_f64(smin);
      fmx = wave_max_f64(fmx);
      gmx = wave_max_f64(gmx);
      mmx = wave_max_f64(mmx);
      if (lane == 0) {
        bsw_max[blk] = smax > 0.0 ? __double2float_ru(smax) : 0.0f;
        bsw_min[blk] = smin < INFINITY ? __double2float_rd(smin) : INFINITY;
        bdf_max[blk] = __double2float_ru(fmx);
        bdg_max[blk] = __double2float_ru(gmx);
        bmu_max[blk] = __double2float_ru(mmx);
      }
    }
  }
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
// Matrix-profile entries at L from the best keys: the FP64 distance of every
// chosen pair is evaluated directly from the z-normalised windows (no closed
// form, exact near d = 0), in a canonical (min, max) order so d(i, j) = d(j, i)
// bit for bit. Also applies Alg. updateVALMP (strictly smaller normalised
// distance wins, so the shorter length keeps ties).
constexpr int kFinG = 8;  // lanes per owner in k_finalize, each summing every kFinG-th term

__global__ __launch_bounds__(128) void k_finalize(const double* __restrict__ xs, const double* __restrict__ mu,
                                                  const double* __restrict__ sig, const uint64_t* __restrict__ best,
                                                  int64_t N, int64_t N0, int L, double* __restrict__ ring_dist,
                                                  int32_t* __restrict__ ring_idx, double* __restrict__ prof_dist,
                                                  int32_t* __restrict__ prof_idx, double* __restrict__ valmp_norm,
                                                  double* __restrict__ valmp_dist, int32_t* __restrict__ valmp_len,
                                                  int32_t* __restrict__ valmp_idx) {
  const int r = threadIdx.x % kFinG;
  const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kFinG;
  const uint64_t key = o < N ? best[o] : kEmptyKey;
  // the group's lanes split the sum of squared differences (adjacent lanes,
  // adjacent terms); every lane reaches the reduction
  double acc = 0.0;
  int64_t c = -1;
  if (key != kEmptyKey) {
    c = key_cand(key);
    const int64_t a = o < c ? o : c, b = o < c ? c : o;
    const double ma = mu[a], mb = mu[b];
    const double ia = 1.0 / sig[a], ib = 1.0 / sig[b];
    for (int k = r; k < L; k += kFinG) {
      const double z = (xs[a + k] - ma) * ia - (xs[b + k] - mb) * ib;
      acc = fma(z, z, acc);
    }
  }
#pragma unroll
  for (int m = kFinG / 2; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, kWave);
  if (r != 0) return;
  if (o >= N) {
    if (o < N0) {  // the row's entries past N_L (no window of this length)
      ring_dist[o] = INFINITY;
      ring_idx[o] = -1;
      if (prof_dist) prof_dist[o] = INFINITY;
      if (prof_idx) prof_idx[o] = -1;
    }
    return;
  }
  const double d = key != kEmptyKey ? sqrt(acc) : INFINITY;
  const int32_t c32 = (int32_t)c;
  ring_dist[o] = d;
  ring_idx[o] = c32;
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
                               int64_t valid, int64_t failed, int recomputed, int64_t passes, int rebuilt) {
  if (threadIdx.x != 0) return;
  if (row) {
    row[0] = valid;
    row[1] = failed;
    row[2] = recomputed == 2 ? (int64_t)cnt[CNT_NREC] : (recomputed ? (int64_t)cnt[CNT_NFAIL] : 0);
    row[3] = full_pass;
    row[4] = (int64_t)cnt[CNT_NFLAT];
    row[5] = (int64_t)cnt[CNT_APPENDS];
    row[6] = (int64_t)cnt[CNT_EV_STEPS];
    row[7] = (int64_t)cnt[CNT_EV_HITS];
    row[8] = (int64_t)cnt[CNT_HARD];
    row[9] = passes;
    row[10] = (int64_t)cnt[CNT_NPART];
    row[11] = (int64_t)cnt[CNT_MCERT];
    row[12] = (int64_t)cnt[CNT_MREC];
    row[13] = (int64_t)cnt[CNT_MPRUNED];
    row[14] = rebuilt ? (int64_t)cnt[CNT_OVER] : 0;  // CNT_OVER is kept until the next rebuild
  }
  cnt[CNT_NFLAT] = cnt[CNT_EV_STEPS] = cnt[CNT_EV_HITS] = cnt[CNT_APPENDS] = 0;
  cnt[CNT_NFAIL] = cnt[CNT_VALID] = cnt[CNT_HARD] = cnt[CNT_BIG] = 0;
  cnt[CNT_NREC] = cnt[CNT_NPART] = cnt[CNT_RFLAT] = 0;
  cnt[CNT_MOPEN] = cnt[CNT_MREC] = cnt[CNT_MCERT] = cnt[CNT_MPRUNED] = 0;
}

__global__ void k_fill_counters(unsigned long long* __restrict__ p, int n, unsigned long long v) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = v;
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

// Endpoints of the accepted pairs, sorted by offset, with each pair's length:
// a test only visits the endpoints within the widest exclusion zone of x.
struct PickSet {
  int32_t pos[2 * kMaxK];
  int32_t len[2 * kMaxK];
  int n;
};

// inserts the two endpoints of an accepted pair (one thread)
__device__ __forceinline__ void pick_insert(PickSet& ps, int32_t a, int32_t b, int32_t L) {
  const int32_t v[2] = {a, b};
  for (int u = 0; u < 2; ++u) {
    int q = ps.n++;
    while (q > 0 && ps.pos[q - 1] > v[u]) {
      ps.pos[q] = ps.pos[q - 1];
      ps.len[q] = ps.len[q - 1];
      --q;
    }
    ps.pos[q] = v[u];
    ps.len[q] = L;
  }
}

// true if offset x lies within the exclusion zone of an accepted endpoint; the
// zone of the pair (x's length Lx, endpoint length Lp) is that of the longer
// length when `longer` is set, else the fixed e; emax bounds every zone
__device__ __forceinline__ bool near_pick(const PickSet& ps, int64_t x, int64_t emax, bool longer, int64_t Lx,
                                          int excl_den, int64_t e) {
  int lo = 0, hi = ps.n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)ps.pos[mid] < x - emax)
      lo = mid + 1;
    else
      hi = mid;
  }
  for (int q = lo; q < ps.n && (int64_t)ps.pos[q] <= x + emax; ++q) {
    const int64_t eq = longer ? excl_zone(Lx > ps.len[q] ? Lx : ps.len[q], excl_den) : e;
    if (iabs64(x - ps.pos[q]) <= eq) return true;
  }
  return false;
}

// Per length t: motif pairs (C14 reading: sort by (d, min, max), greedy with
// the exclusion zone on all four endpoint combinations).
__global__ __launch_bounds__(kRankThreads) void k_topk_motifs(
    const double* __restrict__ prof_dist, const int32_t* __restrict__ prof_idx, int64_t N0,
    int64_t n, int l_min, int excl_den, int k, int32_t* __restrict__ motif_ab, double* __restrict__ motif_d) {
  __shared__ MotifKey sh[kRankThreads];
  __shared__ PickSet ps;
  if (threadIdx.x == 0) ps.n = 0;
  __syncthreads();
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
      if (!near_pick(ps, m.a, e, false, L, excl_den, e) && !near_pick(ps, m.b, e, false, L, excl_den, e)) best = m;
    }
    best = block_reduce(best, motif_less, sh);
    if (!(best.d < INFINITY)) break;
    if (threadIdx.x == 0) {
      pick_insert(ps, best.a, best.b, L);
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
// (lstep = 0: every block ranks a column of one length, e.g. the j-th best-match
// distances of the m-th discords.)
__global__ __launch_bounds__(kRankThreads) void k_topk_discords(
    const double* __restrict__ prof_dist, const int32_t* __restrict__ prof_idx, int64_t N0,
    int64_t n, int l_min, int lstep, int excl_den, int k, int32_t* __restrict__ discord_on,
    double* __restrict__ discord_d, int emul = 1) {
  __shared__ DiscordKey sh[kRankThreads];
  __shared__ int32_t acc_i[kMaxK];
  const int tl = blockIdx.x;
  const int L = l_min + tl * lstep;
  const int64_t N = n - L + 1;
  const int64_t e = emul * excl_zone(L, excl_den);
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
  __shared__ PickSet ps;
  if (threadIdx.x == 0) ps.n = 0;
  __syncthreads();
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
  const int64_t emax = excl_zone(l_min + nlen - 1, excl_den);  // zone of the longest length
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
      if (!near_pick(ps, a, emax, true, m.L, excl_den, 0) && !near_pick(ps, b, emax, true, m.L, excl_den, 0))
        best = m;
    }
    best = block_reduce(best, gmotif_less, sh);
    if (!(best.dn < INFINITY)) break;
    if (threadIdx.x == 0) {
      const int32_t i = best.i, c = valmp_idx[i];
      const int32_t a = i < c ? i : c, b = i < c ? c : i;
      pick_insert(ps, a, b, best.L);
      g_motif_abl[got * 3] = a;
      g_motif_abl[got * 3 + 1] = b;
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

hipError_t launch_window_prep(const WindowPrep& w, hipStream_t st) {
  const unsigned blocks = blocks_for(w.N + kPad, 256);
  if (w.hflat && (!w.hsig || !w.rflat)) return hipErrorInvalidValue;
  if (w.bsw_max && (!w.bsw_min || !w.bdf_max || !w.bdg_max || !w.bmu_max)) return hipErrorInvalidValue;
  if (w.df32)
    k_window_prep<true><<<blocks, 256, 0, st>>>(w.xs, w.N, w.L, w.first, w.flat_eps, w.A_in, w.B_in, w.A_out, w.B_out,
                                                w.mu, w.sig, w.invn, w.flat, w.nflat, w.df, w.dg, w.sw32, w.df32,
                                                w.dg32, w.inv32, w.bsw_max, w.bsw_min, w.bdf_max, w.bdg_max,
                                                w.bmu_max, w.hflat, w.hsig, w.rflat);
  else
    k_window_prep<false><<<blocks, 256, 0, st>>>(w.xs, w.N, w.L, w.first, w.flat_eps, w.A_in, w.B_in, w.A_out,
                                                 w.B_out, w.mu, w.sig, w.invn, w.flat, w.nflat, w.df, w.dg, w.sw32,
                                                 nullptr, nullptr, nullptr, w.bsw_max, w.bsw_min, w.bdf_max,
                                                 w.bdg_max, w.bmu_max, w.hflat, w.hsig, w.rflat);
  return hipGetLastError();
}

hipError_t launch_seed_mp(const double* xs, const double* mu, const double* invn, const uint8_t* flat,
                          const int32_t* prev_idx, int64_t N, int L, int64_t e, uint64_t* best,
                          double* thr, float* thr32, hipStream_t st) {
  k_seed_mp<<<blocks_for(N + kPad, 128), 128, 0, st>>>(xs, mu, invn, flat, prev_idx, N, L, e, best, thr, thr32);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* xs, const double* mu, const double* sig, const uint64_t* best,
                           int64_t N, int64_t N0, int L, double* ring_dist, int32_t* ring_idx, double* prof_dist,
                           int32_t* prof_idx, double* valmp_norm, double* valmp_dist, int32_t* valmp_len,
                           int32_t* valmp_idx, hipStream_t st) {
  if (!ring_dist || !ring_idx) return hipErrorInvalidValue;
  const int64_t n = N0 > N ? N0 : N;
  k_finalize<<<blocks_for(n * kFinG, 128), 128, 0, st>>>(xs, mu, sig, best, N, N0, L, ring_dist, ring_idx, prof_dist,
                                                         prof_idx, valmp_norm, valmp_dist, valmp_len, valmp_idx);
  return hipGetLastError();
}

hipError_t launch_record_stats(unsigned long long* cnt, int64_t* row, int full_pass, int64_t valid,
                               int64_t failed, int recomputed, int64_t passes, int rebuilt, hipStream_t st) {
  k_record_stats<<<1, 64, 0, st>>>(cnt, row, full_pass, valid, failed, recomputed, passes, rebuilt);
  return hipGetLastError();
}

hipError_t launch_fill_counters(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
  if (n <= 0 || n > 64) return hipErrorInvalidValue;
  k_fill_counters<<<1, 64, 0, st>>>(p, n, v);
  return hipGetLastError();
}

__global__ void k_keys_to_idx(const uint64_t* __restrict__ best, int64_t N, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint64_t k = best[i];
  idx[i] = k == kEmptyKey ? -1 : (int32_t)key_cand(k);
}

hipError_t launch_keys_to_idx(const uint64_t* best, int64_t N, int32_t* idx, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_keys_to_idx<<<blocks_for(N, 256), 256, 0, st>>>(best, N, idx);
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
    k_topk_discords<<<nlen, kRankThreads, 0, st>>>(prof_dist, prof_idx, N0, n, l_min, 1, excl_den, kd, discord_on,
                                                   discord_d);
  return hipGetLastError();
}

// m-th discords of one length: columns j = 0..m-1 of vals / nn (stride N0)
hipError_t launch_mth_rankings(const double* vals, const int32_t* nn, int64_t N0, int64_t n, int L, int m,
                               int excl_den, int kd, int32_t* on, double* d, hipStream_t st, int emul) {
  if (m <= 0 || kd <= 0 || kd > kMaxK || emul < 1) return hipErrorInvalidValue;
  k_topk_discords<<<m, kRankThreads, 0, st>>>(vals, nn, N0, n, L, 0, excl_den, kd, on, d, emul);
  return hipGetLastError();
}

// Cross-length m-th discords (Alg. UpdateVariableLengthDiscords): for each
// (j, rank), the largest d / sqrt(L) over the lengths, strictly (shorter wins ties).
__global__ void k_mth_global(const int32_t* __restrict__ on, const double* __restrict__ d, int nlen, int l_min,
                             int m, int kd, int32_t* __restrict__ g_onl, double* __restrict__ g_d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;  // q = j * kd + r
  if (q >= m * kd) return;
  const int j = q / kd, r = q % kd;
  double best = -INFINITY, db = NAN, dnb = NAN;
  int32_t o = -1, nb = -1, Lb = -1;
  for (int t = 0; t < nlen; ++t) {
    const int64_t at = ((int64_t)t * m + j) * kd + r;
    const double v = d[at];
    if (!(v == v)) continue;
    const int L = l_min + t;
    const double dn = v / sqrt((double)L);
    if (dn > best) {
      best = dn;
      db = v;
      dnb = dn;
      o = on[at * 2];
      nb = on[at * 2 + 1];
      Lb = L;
    }
  }
  g_onl[q * 3] = o;
  g_onl[q * 3 + 1] = nb;
  g_onl[q * 3 + 2] = Lb;
  g_d[q * 2] = db;
  g_d[q * 2 + 1] = dnb;
}

hipError_t launch_mth_global(const int32_t* on, const double* d, int nlen, int l_min, int m, int kd,
                             int32_t* g_onl, double* g_d, hipStream_t st) {
  if (m * kd <= 0) return hipSuccess;
  k_mth_global<<<blocks_for(m * kd, 64), 64, 0, st>>>(on, d, nlen, l_min, m, kd, g_onl, g_d);
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
