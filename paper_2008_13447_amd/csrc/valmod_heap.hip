// Partial distance profiles of VALMOD (gfx950): thresholds for the collecting
// pass, the exact merge into top-p partial profiles, the per-length sweep with
// the lower-bound test (Alg. ComputeSubMP) and the exact row recompute of the
// windows whose test fails.
//
// A partial profile of owner o at base length b holds up to p candidates with
// the largest base-length correlation (the p smallest lower bounds, Eq.
// lowerBoundFinalFormula) together with the anchored cross sum
//   S_L(o, c) = sum_{k<L} (x_{o+k} - x_o) (x_{c+k} - x_c),
// which grows by one term per length, so the exact correlation at any later L
// costs O(1): rho_L = (S_L - A_o A_c / L) / (L sigma_o sigma_c), with A the
// anchored window sums of the statistics kernel. Every candidate not stored has
// a base correlation <= bound_rho (stored per owner), hence a distance at L of
// at least sqrt(b (1 - max(bound_rho, 0)^2)) sigma_{o,b} / sigma_{o,L}
// (Eq. lowerBoundFinalFormula), except the windows that were flat at b (never
// collected): each of them, c, is at least sqrt(b) (sigma_{o,b} / sigma_{o,L} -
// sigma_{c,b} / sigma_{c,L}) away, and the sweep takes the smaller bound.
#include "valmod_common.h"
#include "valmod_kernels.h"

#include <math.h>

namespace valmod {

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// anchored cross sum of windows o and c at length L (direct, L - 1 FMAs in
// order of k; the loads of 8 terms are issued before their FMAs)
__device__ __forceinline__ double cross_sum(const double* __restrict__ xs, int L, int64_t o, int64_t c) {
  const double xo = xs[o], xc = xs[c];
  double s = 0.0;
  int k = 1;
  for (; k + 8 <= L; k += 8) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = xs[o + k + u];
      b[u] = xs[c + k + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s = fma(a[u] - xo, b[u] - xc, s);
  }
  for (; k < L; ++k) s = fma(xs[o + k] - xo, xs[c + k] - xc, s);
  return s;
}

// the terms k in [kb, ke) of the anchored cross sum (a chunk of cross_sum)
__device__ __forceinline__ double cross_sum_range(const double* __restrict__ xs, int64_t o, int64_t c, int kb,
                                                  int ke) {
  const double xo = xs[o], xc = xs[c];
  double s = 0.0;
  int k = kb;
  for (; k + 8 <= ke; k += 8) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = xs[o + k + u];
      b[u] = xs[c + k + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s = fma(a[u] - xo, b[u] - xc, s);
  }
  for (; k < ke; ++k) s = fma(xs[o + k] - xo, xs[c + k] - xc, s);
  return s;
}

__device__ __forceinline__ double rho_from_sum(double S, double Ao, double Ac, int L, double io, double ic) {
  return (S - Ao * Ac / (double)L) * io * ic;
}

__device__ __forceinline__ void push_fail(int32_t* fail, unsigned long long* nfail, int64_t o) {
  const unsigned long long pos = atomicAdd(nfail, 1ull);
  fail[pos] = (int32_t)o;
}

// wavefront-aggregated push: one atomic per wavefront for every lane with `want`
__device__ __forceinline__ void push_fail_wave(bool want, int32_t* fail, unsigned long long* nfail, int64_t o) {
  const uint64_t m = __ballot(want);
  if (!m) return;
  const int lane = (int)__lane_id();
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(nfail, (unsigned long long)__popcll(m));
  base = shfl_u64(base, leader);
  if (want) fail[base + __popcll(m & ((uint64_t(1) << lane) - 1))] = (int32_t)o;
}

__device__ __forceinline__ void count_wave(bool want, unsigned long long* counter) {
  const uint64_t m = __ballot(want);
  if (!m) return;
  if ((int)__lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(counter, (unsigned long long)__popcll(m));
}

// number of active lanes whose 64-bit key is smaller than `key`
__device__ __forceinline__ int wave_rank(uint64_t key, bool valid) {
  int r = 0;
  for (int m = 0; m < kWave; ++m) {
    const uint64_t other = shfl_u64(key, m);
    const int ov = __shfl((int)valid, m, kWave);
    r += (ov && other < key) ? 1 : 0;
  }
  return r;
}

// --------------------------------------------------------------------------
// Thresholds of the collecting pass. For owner o the candidates
//   src[o + d] - d (|d| <= D: the neighbour of a nearby window carried along
//   the diagonal) and src[o] + d (|d| <= D: around its own neighbour)
// are evaluated exactly; with m distinct eligible candidates the threshold is
// the min(p, m)-th largest correlation, which is at most the true p-th largest
// (and at most the true largest), lowered by a margin covering the rounding of
// the pass. Owners with no eligible candidate collect nothing and go to the
// recompute list. A group of G >= 4D + 2 lanes per owner (one lane for D = 0,
// the single candidate src[o]).
template <int G>
__global__ __launch_bounds__(kWave) void k_seed_append(const double* __restrict__ xs, const double* __restrict__ A,
                                                       const double* __restrict__ invn,
                                                       const uint8_t* __restrict__ flat,
                                                       const int32_t* __restrict__ src, int64_t N, int L, int64_t e,
                                                       int p, int D, double margin, int best_exact,
                                                       double* __restrict__ thr, float* __restrict__ thr32,
                                                       uint32_t* __restrict__ cnt, int32_t* __restrict__ fail,
                                                       unsigned long long* __restrict__ nfail) {
  auto set_thr = [&](int64_t w, double v) {
    thr[w] = v;
    if (thr32) thr32[w] = __double2float_rd(v);
  };
  constexpr int OPW = kWave / G;  // owners per wavefront
  const int t = threadIdx.x, l = t % G, gb = t - l;
  const int64_t o = (int64_t)blockIdx.x * OPW + t / G;
  const bool live = o < N;
  const bool fl = live ? flat[o] != 0 : true;
  int64_t c = -1;
  if (!fl) {
    if (l <= 2 * D) {
      const int64_t d = l - D, w = o + d;
      if (w >= 0 && w < N && src[w] >= 0) c = (int64_t)src[w] - d;
    } else if (l <= 4 * D + 1) {
      const int64_t d = l - (3 * D + 1);
      if (src[o] >= 0) c = (int64_t)src[o] + d;
    }
  }
  bool ok = c >= 0 && c < N && iabs64(c - o) > e && !flat[c];
  // drop duplicates: keep the lowest lane of the group holding each candidate
  for (int m = 0; m < G; ++m) {
    const int64_t oc = (int64_t)__shfl((int)c, gb + m, kWave);
    const int ov = __shfl((int)ok, gb + m, kWave);
    if (m < l && ov && oc == c) ok = false;
  }
  uint64_t key = kEmptyKey;
  double rho = -2.0;
  if (ok) {
    rho = rho_from_sum(cross_sum(xs, L, o, c), A[o], A[c], L, invn[o], invn[c]);
    key = make_key(rho, c);
  }
  int mg = 0, rank = 0;  // eligible candidates of the group, and this lane's rank among them
  for (int m = 0; m < G; ++m) {
    const uint64_t other = shfl_u64(key, gb + m);
    const int ov = __shfl((int)ok, gb + m, kWave);
    mg += ov;
    rank += (ov && other < key) ? 1 : 0;
  }
  if (!live) return;
  if (l == 0) cnt[o] = 0;
  if (fl) {
    if (l == 0) set_thr(o, 3.0);  // not an owner
    return;
  }
  if (mg == 0) {
    if (l == 0) {
      set_thr(o, 3.0);
      if (!best_exact) push_fail(fail, nfail, o);
    }
    return;
  }
  if ((int64_t)p >= N - 1) {
    if (l == 0) set_thr(o, -2.0 - margin);  // a profile can hold every candidate: collect them all
    return;
  }
  const int want = (p < mg ? p : mg) - 1;
  if (ok && rank == want) set_thr(o, rho - margin);
}

// --------------------------------------------------------------------------
// Merge of the collected candidates into the partial profile of each owner at
// the new base length L: exact correlation of every candidate the pass
// appended, top-`keep` by (correlation desc, index asc), the bound correlation
// of the ones not kept, and the owner's best key. Owners that collected nothing
// go to the recompute list with an empty profile; so do owners whose list
// overflowed (incomplete), which keep the best `keep` of their listed
// candidates as a profile whose bound certifies nothing (k_merge_big), or an
// empty one when keep = 0.
//
// best_exact: `best` already holds every owner's exact neighbour (a
// matrix-profile pass ran at this length), so an owner whose profile cannot be
// built keeps it instead of going to the recompute list.
//
// k_merge_small takes a group of kSmallG lanes per owner and up to kSmallG
// candidates (the group's lanes split the terms of the candidates' sums when
// there are fewer); owners with more candidates are listed for k_merge_big (one
// wavefront per owner, candidates in LDS).
constexpr int kMergeCap = 512;
constexpr int kSmallG = 8;

// every candidate not collected has an exact correlation below the threshold
// (the pass compares with the threshold lowered by its item's rounding bound);
// below -1 every candidate was collected, and -3 marks a complete profile
__device__ __forceinline__ double collect_bound(double thr, double margin) {
  return thr < -1.5 ? -3.0 : thr + 2.0 * margin;
}

__global__ __launch_bounds__(kWave) void k_merge_small(
    const double* __restrict__ xs, const double* __restrict__ A, const double* __restrict__ invn,
    const double* __restrict__ sig, const uint8_t* __restrict__ flat, const double* __restrict__ thr,
    const uint32_t* __restrict__ cnt, const int32_t* __restrict__ buf, int64_t cap, int64_t N, int L, int p,
    int keep, double margin, int best_exact, int32_t* __restrict__ hc, double* __restrict__ hS, int32_t* __restrict__ hn,
    double* __restrict__ hbound, double* __restrict__ hsig, uint8_t* __restrict__ hflat, uint64_t* __restrict__ best,
    int32_t* __restrict__ fail, unsigned long long* __restrict__ nfail, int32_t* __restrict__ big,
    unsigned long long* __restrict__ nbig, unsigned long long* __restrict__ nover) {
  const int t = threadIdx.x, l = t % kSmallG, gb = t - l;
  const int64_t o = (int64_t)blockIdx.x * (kWave / kSmallG) + t / kSmallG;
  const bool live = o < N;
  int64_t m = 0;
  bool skip = true;
  if (live) {
    m = cnt[o];
    skip = flat[o] || thr[o] >= 2.0;  // not an owner, or already queued for recompute by the seeding
  }
  // the list holds min(m, cap) entries: an owner with more (overflow) is not
  // merged, and its entries past cap are not read (they are another owner's)
  const bool merged = live && !skip && m >= 1 && m <= kSmallG && m <= cap;
  const bool ok = merged && l < m;
  // the group's lanes share the candidates' sums: R = 8 / P lanes per candidate
  // (P = m rounded up to a power of two), each summing a chunk of the terms
  const int P = m <= 1 ? 1 : (m <= 2 ? 2 : (m <= 4 ? 4 : 8));
  const int R = kSmallG / P;
  double part = 0.0;
  if (merged) {
    const int ci = l / R, r = l % R;
    if (ci < m) {
      const int kb = 1 + (int)((int64_t)(L - 1) * r / R), ke = 1 + (int)((int64_t)(L - 1) * (r + 1) / R);
      part = cross_sum_range(xs, o, (int64_t)buf[o * cap + ci], kb, ke);
    }
  }
#pragma unroll
  for (int msk = kSmallG / 2; msk >= 1; msk >>= 1) {
    const double v = __shfl_xor(part, msk, kWave);
    if (msk < R) part += v;
  }
  const double Sg = __shfl(part, gb + (l * R < kSmallG ? l * R : 0), kWave);  // candidate l's sum
  int64_t c = -1;
  double rho = -2.0, S = 0.0;
  uint64_t key = kEmptyKey;
  if (ok) {
    c = buf[o * cap + l];
    S = Sg;
    rho = rho_from_sum(S, A[o], A[c], L, invn[o], invn[c]);
    key = make_key(rho, c);
  }
  int rank = 0;  // keys of the group are distinct; empty keys sort last
  for (int mm = 0; mm < kSmallG; ++mm) rank += shfl_u64(key, gb + mm) < key ? 1 : 0;
  double nb = (ok && rank == keep) ? rho : -4.0;  // the best collected candidate not kept
#pragma unroll
  for (int msk = kSmallG / 2; msk >= 1; msk >>= 1) nb = fmax(nb, __shfl_xor(nb, msk, kWave));
  if (nover) count_wave(live && !skip && m > cap && keep > 0 && l == 0, nover);
  if (!live) return;
  if (skip || m == 0 || (m > cap && keep == 0)) {
    // no partial profile: an empty one whose bound is 0 (bound correlation 1),
    // so that the sweep of a later length never certifies from stale data
    if (l == 0) {
      hn[o] = 0;
      hbound[o] = 2.0;
      hsig[o] = sig[o];
      hflat[o] = flat[o];
      if (skip) {
        if (!best_exact || flat[o]) best[o] = kEmptyKey;
      } else if (!best_exact) {
        best[o] = kEmptyKey;
        push_fail(fail, nfail, o);
      }
    }
    return;
  }
  if (m > cap) {
    // overflow: the list holds the first cap candidates collected, not the best
    // ones. The exact neighbour comes from elsewhere (best_exact) or the recompute
    // list; k_merge_big keeps the best p of the cap as a profile that no sweep
    // certifies (bound correlation 1) but whose candidates give a later rebuild
    // its thresholds (any p real candidates bound the p-th best from below)
    if (l == 0) {
      hflat[o] = 0;
      if (!best_exact) {
        best[o] = kEmptyKey;
        push_fail(fail, nfail, o);
      }
      const unsigned long long pos = atomicAdd(nbig, 1ull);
      if ((int64_t)pos < N) big[pos] = (int32_t)o;
    }
    return;
  }
  if (m > kSmallG) {
    if (l == 0) {
      hflat[o] = 0;  // a non-flat owner (k_merge_big writes the rest)
      // the list holds each owner at most once per merge (its counter is cleared
      // before every collecting pass); never write past its N entries
      const unsigned long long pos = atomicAdd(nbig, 1ull);
      if ((int64_t)pos < N) big[pos] = (int32_t)o;
    }
    return;
  }
  if (ok && rank < keep) {
    hc[o * p + rank] = (int32_t)c;
    hS[o * p + rank] = S;
  }
  if (ok && rank == 0) best[o] = key;
  if (l == 0) {
    // the best candidate not kept was evaluated directly (error <= margin)
    const double sb = collect_bound(thr[o], margin), nbu = nb + margin;
    hn[o] = (int32_t)(m < keep ? m : keep);
    hbound[o] = nbu > sb ? nbu : sb;
    hsig[o] = sig[o];
    hflat[o] = 0;
  }
}

__global__ __launch_bounds__(kWave) void k_merge_big(
    const double* __restrict__ xs, const double* __restrict__ A, const double* __restrict__ invn,
    const double* __restrict__ sig, const double* __restrict__ thr, const uint32_t* __restrict__ cnt,
    const int32_t* __restrict__ buf, int64_t cap, int64_t N, int L, int p, int keep, double margin,
    int32_t* __restrict__ hc, double* __restrict__ hS, int32_t* __restrict__ hn, double* __restrict__ hbound,
    double* __restrict__ hsig, uint64_t* __restrict__ best, const int32_t* __restrict__ big,
    const unsigned long long* __restrict__ nbig) {
  extern __shared__ double merge_lds[];  // cap entries each of key, correlation and cross sum
  uint64_t* skey = (uint64_t*)merge_lds;
  double* srho = merge_lds + cap;
  double* ssum = merge_lds + 2 * cap;
  __shared__ double sbound;
  const int t = threadIdx.x;
  const int64_t listed = (int64_t)*nbig;
  const int64_t count = listed < N ? listed : N;  // the list has N entries
  for (int64_t w = blockIdx.x; w < count; w += gridDim.x) {
    const int64_t o = big[w];
    const int64_t mc = cnt[o];        // kSmallG < mc <= cap, or an overflowed list (mc > cap)
    const bool over = mc > cap;       // the list holds its first cap candidates
    const int64_t m = over ? cap : mc;
    const double Ao = A[o], io = invn[o];
    const int32_t* list = buf + o * cap;
    for (int64_t r = t; r < m; r += kWave) {
      const int64_t c = list[r];
      const double S = cross_sum(xs, L, o, c);
      const double rho = rho_from_sum(S, Ao, A[c], L, io, invn[c]);
      skey[r] = make_key(rho, c);
      srho[r] = rho;
      ssum[r] = S;
    }
    if (t == 0) sbound = collect_bound(thr[o], margin);
    __syncthreads();
    for (int64_t r = t; r < m; r += kWave) {
      const uint64_t k = skey[r];
      int64_t rank = 0;
      for (int64_t s2 = 0; s2 < m; ++s2) rank += skey[s2] < k ? 1 : 0;
      if (rank < keep) {
        hc[o * p + rank] = (int32_t)key_cand(k);
        hS[o * p + rank] = ssum[r];
      }
      if (rank == 0 && !over) best[o] = k;
      if (rank == keep && srho[r] + margin > sbound) sbound = srho[r] + margin;  // a single lane has this rank
    }
    __syncthreads();
    if (t == 0) {
      hn[o] = (int32_t)(m < keep ? m : keep);
      hbound[o] = over ? 2.0 : sbound;  // overflowed: candidates outside the list are unbounded
      hsig[o] = sig[o];
    }
    __syncthreads();  // the LDS lists are reused by the next owner
  }
}

// Lower bound at L of the distance from owner o to every candidate its partial
// profile (built at the base length b) does not hold (Eq. lowerBoundFinalFormula,
// rescaled by sigma_{o,b} / sigma_{o,L} as in Alg. ComputeSubMP): +inf for a
// complete profile, 0 for an owner without a profile. rf > 0: the largest
// sigma_b / sigma_L of the windows flat at b (never stored) that are candidates
// at L, which bounds those from below as well.
__device__ __forceinline__ double unstored_bound(int64_t o, int base, const double* __restrict__ sig,
                                                 const double* __restrict__ hbound, const double* __restrict__ hsig,
                                                 double rf) {
  if (!(hsig[o] > 0.0)) return 0.0;
  const double ro = hsig[o] / sig[o];  // sigma_{o,b} / sigma_{o,L}
  double lb;
  if (hbound[o] < -2.5) {
    lb = INFINITY;  // complete profile: no candidate was left out
  } else {
    const double q = hbound[o] > 0.0 ? (hbound[o] < 1.0 ? hbound[o] : 1.0) : 0.0;
    lb = sqrt((double)base * (1.0 - q * q)) * ro;
  }
  if (rf > 0.0) {
    const double lbf = sqrt((double)base) * (ro > rf ? ro - rf : 0.0);
    lb = lbf < lb ? lbf : lb;
  }
  return lb;
}

// --------------------------------------------------------------------------
// Per-length sweep (Alg. ComputeSubMP): grow every stored cross sum by one
// term, take the exact minimum over the stored candidates still eligible at L,
// and certify it against the lower bound of the candidates not stored (rank
// preservation: the bound only rescales by sigma_{o,b} / sigma_{o,L}). Certified
// owners get their best key; the others go to the recompute list. One thread
// per owner.
__global__ void k_sweep(const double* __restrict__ xs, const double* __restrict__ A, const double* __restrict__ invn,
                        const double* __restrict__ sig, const uint8_t* __restrict__ flat, int64_t N, int L, int64_t e,
                        int p, int base, const int32_t* __restrict__ hc, double* __restrict__ hS,
                        const int32_t* __restrict__ hn, const double* __restrict__ hbound,
                        const double* __restrict__ hsig, const unsigned long long* __restrict__ rflat, double margin,
                        uint64_t* __restrict__ best, int32_t* __restrict__ fail,
                        unsigned long long* __restrict__ nfail, unsigned long long* __restrict__ nvalid,
                        double* __restrict__ lbm, unsigned long long* __restrict__ min_dist,
                        unsigned long long* __restrict__ min_lb) {
  // lbm / min_dist / min_lb (optional, Alg. ComputeSubMP's bookkeeping): the
  // bound of every failing owner, and the minima over the owners of the certified
  // distances (minDistAbs) and of the failing owners' bounds (minLbAbs), as the
  // bit patterns of non-negative doubles (ordered like the values).
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = o < N;
  const bool owner = live && !flat[o];
  if (live && !owner) best[o] = kEmptyKey;
  bool valid = false;
  double min_d = INFINITY, max_lb = 0.0;
  uint64_t kb = kEmptyKey;
  double rb = -2.0;
  if (live) {
    // every stored sum grows to L, also those of an owner flat at this length
    // (one that is not flat at a later length reads them again)
    const int nh = hn[o];
    const double xo = xs[o], dx = xs[o + L - 1] - xo;
    const double Ao = A[o], io = invn[o];
    for (int r = 0; r < nh; ++r) {
      const int64_t c = hc[o * p + r];
      if (c >= N) continue;  // no window of length L at c (nor at any longer length)
      const double S = fma(dx, xs[c + L - 1] - xs[c], hS[o * p + r]);
      hS[o * p + r] = S;
      if (!owner || iabs64(c - o) <= e || flat[c]) continue;
      const double rho = rho_from_sum(S, Ao, A[c], L, io, invn[c]);
      const uint64_t k = make_key(rho, c);
      if (k < kb) {
        kb = k;
        rb = rho;
      }
    }
  }
  if (owner) {
    max_lb = unstored_bound(o, base, sig, hbound, hsig, __longlong_as_double((long long)*rflat));
    if (kb != kEmptyKey) {
      // the stored minimum from a correlation evaluated directly (error <= margin):
      // certified when even its largest possible exact distance is below the bound
      const double u = 1.0 - rb;
      min_d = sqrt(2.0 * (double)L * (u > 0.0 ? u : 0.0));
      const double uh = u + margin;
      const double d_hi = sqrt(2.0 * (double)L * (uh > 0.0 ? uh : 0.0));
      valid = hsig[o] > 0.0 && (max_lb == INFINITY || d_hi < max_lb * (1.0 - 1.0e-12));
    }
    best[o] = valid ? kb : kEmptyKey;
    if (!valid && lbm) lbm[o] = max_lb < INFINITY ? max_lb : 0.0;
  }
  count_wave(valid, nvalid);
  push_fail_wave(owner && !valid, fail, nfail, o);
  if (min_dist) {
    uint64_t a = valid ? (uint64_t)__double_as_longlong(min_d) : kEmptyKey;
    uint64_t b = (owner && !valid && max_lb < INFINITY) ? (uint64_t)__double_as_longlong(max_lb) : kEmptyKey;
    a = wave_min_u64(a);
    b = wave_min_u64(b);
    if ((threadIdx.x % kWave) == 0) {
      if (a != kEmptyKey) atomicMin(min_dist, (unsigned long long)a);
      if (b != kEmptyKey) atomicMin(min_lb, (unsigned long long)b);
    }
  }
}

// Alg. ComputeSubMP after a failed bound test: the failing owners whose bound is
// below the best certified distance (`limit`, bits of a non-negative double) are
// listed for the row recompute; the others stay partial (their profile entry is
// not computed at this length).
__global__ void k_split_fail(const int32_t* __restrict__ fail, const unsigned long long* __restrict__ nfail,
                             const double* __restrict__ lbm, const unsigned long long* __restrict__ limit,
                             int all_partial, int32_t* __restrict__ rec, unsigned long long* __restrict__ nrec,
                             int32_t* __restrict__ part, unsigned long long* __restrict__ npart) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t count = (int64_t)*nfail;
  const bool live = w < count;
  const int64_t o = live ? fail[w] : 0;
  const double lim = __longlong_as_double((long long)*limit);
  const bool r = live && !all_partial && lbm[o] < lim;
  push_fail_wave(r, rec, nrec, o);
  push_fail_wave(live && !r, part, npart, o);
}

// Partial entries: index -2 and, as distance, the lower bound of the entry.
__global__ void k_mark_partial(const int32_t* __restrict__ part, const unsigned long long* __restrict__ npart,
                               const double* __restrict__ lbm, double* __restrict__ prof_dist,
                               int32_t* __restrict__ prof_idx) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= (int64_t)*npart) return;
  const int64_t o = part[w];
  if (prof_dist) prof_dist[o] = lbm[o];
  if (prof_idx) prof_idx[o] = -2;
}

// --------------------------------------------------------------------------
// Exact row recompute of the listed owners: the whole distance profile at L
// (every eligible candidate, anchored cross sums formed directly), reduced to
// the best key. The candidates of one owner are spread over gridDim.x
// workgroups, kRecK consecutive candidates per lane sharing one sliding
// register window; the partial minima meet in a 64-bit atomic min on a key
// that the listing kernel has set to empty.
constexpr int kRecK = 8;


__global__ __launch_bounds__(kWave) void k_recompute(const double* __restrict__ xs, const double* __restrict__ A,
                                                     const double* __restrict__ invn,
                                                     const uint8_t* __restrict__ flat,
                                                     const int32_t* __restrict__ fail,
                                                     const unsigned long long* __restrict__ nfail, int64_t N, int L,
                                                     int64_t e, uint64_t* __restrict__ best) {
  const int64_t count = (int64_t)*nfail;
  const int t = threadIdx.x;
  const int64_t c0 = ((int64_t)blockIdx.x * kWave + t) * kRecK;
  for (int64_t w = blockIdx.y; w < count; w += gridDim.y) {
    const int64_t o = fail[w];
    uint64_t kb = kEmptyKey;
    if (c0 < N && !flat[o]) {
      double S[kRecK];
      direct_sums_ahead<kRecK>(xs, o, c0, L, S);
      const double Ao = A[o], io = invn[o];
#pragma unroll
      for (int q = 0; q < kRecK; ++q) {
        const int64_t c = c0 + q;
        if (c >= N || iabs64(c - o) <= e || flat[c]) continue;
        const uint64_t k = make_key(rho_from_sum(S[q], Ao, A[c], L, io, invn[c]), c);
        kb = k < kb ? k : kb;
      }
    }
    kb = wave_min_u64(kb);
    if (t == 0 && kb != kEmptyKey) atomicMin((unsigned long long*)&best[o], (unsigned long long)kb);
  }
}


// total of per-owner counts (one atomic per workgroup)
__global__ __launch_bounds__(1024) void k_sum_counts(const uint32_t* __restrict__ v, int64_t n,
                                                     unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[1024 / kWave];
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += v[i];
#pragma unroll
  for (int m = kWave / 2; m >= 1; m >>= 1) acc += shfl_xor_u64(acc, m);
  if (__lane_id() == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += part[w];
    if (s) atomicAdd(out, s);
  }
}

// --------------------------------------------------------------------------
// Top-m row recompute (m-th best matches of the listed owners): round j keeps,
// for each listed owner, the smallest key strictly above the owner's key of
// round j - 1, so m rounds give the m best candidates in key order. Same
// decomposition as k_recompute; out[o * m + j] must be empty before round j.
__global__ __launch_bounds__(kWave) void k_recompute_round(const double* __restrict__ xs, const double* __restrict__ A,
                                                           const double* __restrict__ invn,
                                                           const uint8_t* __restrict__ flat,
                                                           const int32_t* __restrict__ fail,
                                                           const unsigned long long* __restrict__ nfail, int64_t N,
                                                           int L, int64_t e, int m, int j,
                                                           uint64_t* __restrict__ keys) {
  const int64_t count = (int64_t)*nfail;
  const int t = threadIdx.x;
  const int64_t c0 = ((int64_t)blockIdx.x * kWave + t) * kRecK;
  for (int64_t w = blockIdx.y; w < count; w += gridDim.y) {
    const int64_t o = fail[w];
    const uint64_t floor_key = j > 0 ? keys[o * m + j - 1] : 0;
    uint64_t kb = kEmptyKey;
    if (c0 < N && !flat[o] && (j == 0 || floor_key != kEmptyKey)) {
      double S[kRecK];
      direct_sums_ahead<kRecK>(xs, o, c0, L, S);
      const double Ao = A[o], io = invn[o];
#pragma unroll
      for (int q = 0; q < kRecK; ++q) {
        const int64_t c = c0 + q;
        if (c >= N || iabs64(c - o) <= e || flat[c]) continue;
        const uint64_t k = make_key(rho_from_sum(S[q], Ao, A[c], L, io, invn[c]), c);
        if (j > 0 && k <= floor_key) continue;
        kb = k < kb ? k : kb;
      }
    }
    kb = wave_min_u64(kb);
    if (t == 0 && kb != kEmptyKey) atomicMin((unsigned long long*)&keys[o * m + j], (unsigned long long)kb);
  }
}

// empties the m keys of every listed owner
__global__ void k_clear_keys(const int32_t* __restrict__ fail, const unsigned long long* __restrict__ nfail, int m,
                             uint64_t* __restrict__ keys) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= (int64_t)*nfail) return;
  const int64_t o = fail[w];
  for (int j = 0; j < m; ++j) keys[o * m + j] = kEmptyKey;
}

// the recomputed lists become the owners' top-m lists (anchored sums formed directly)
__global__ void k_topm_store(const double* __restrict__ xs, const int32_t* __restrict__ fail,
                             const unsigned long long* __restrict__ nfail, int L, int m, int p,
                             const uint64_t* __restrict__ keys, int32_t* __restrict__ hc, double* __restrict__ hS,
                             int32_t* __restrict__ hn, uint64_t* __restrict__ best) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= (int64_t)*nfail) return;
  const int64_t o = fail[w];
  int cnt = 0;
  for (int j = 0; j < m; ++j) {
    const uint64_t k = keys[o * m + j];
    if (k == kEmptyKey) break;
    const int64_t c = key_cand(k);
    hc[o * p + j] = (int32_t)c;
    hS[o * p + j] = cross_sum(xs, L, o, c);
    ++cnt;
  }
  hn[o] = cnt;
  best[o] = keys[o * m];
}

// j-th best-match distances of every owner from its exact top-m list
// (d = sqrt(2 L (1 - rho)), Eq. 6), column-major: vals[j * N0 + o]
__global__ void k_mth_values(const double* __restrict__ A, const double* __restrict__ invn,
                             const uint8_t* __restrict__ flat, const int32_t* __restrict__ hc,
                             const double* __restrict__ hS, const int32_t* __restrict__ hn, int p, int m, int64_t N,
                             int64_t N0, int L, double* __restrict__ vals, int32_t* __restrict__ nn) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  const int cnt = flat[o] ? 0 : hn[o];
  for (int j = 0; j < m; ++j) {
    double d = INFINITY;
    int32_t c = -1;
    if (j < cnt) {
      c = hc[o * p + j];
      const double rho = rho_from_sum(hS[o * p + j], A[o], A[c], L, invn[o], invn[c]);
      const double u = 1.0 - rho;
      d = sqrt(2.0 * (double)L * (u > 0.0 ? u : 0.0));
    }
    vals[(int64_t)j * N0 + o] = d;
    nn[(int64_t)j * N0 + o] = c;
  }
}

// --------------------------------------------------------------------------
// Top-k m-th discords from the partial profiles (Alg. Topkm_nextLength).
//
// k_mth_select, one thread per owner at length L: the m best stored candidates in
// key order (m rounds over the stored list) and whether they are the owner's
// exact m best matches, i.e. the m-th one's largest possible distance lies below
// the bound of the unstored candidates (a complete profile also certifies fewer
// than m). Certified owners get their j-th best-match distances in vals / nn
// (column j, stride N0). The others get no entry (nn = -1) and, in ub, upper
// bounds of those distances: the j-th stored candidate's distance widened by two
// correlation error margins (its stored sum, and a later direct evaluation), or
// +inf. Any m real candidates bound the m best matches from above, so this also
// holds for an owner whose collecting list overflowed at a rebuild (`fresh`: the
// profiles were rebuilt at this length; such an owner stores the best of its
// listed candidates, and its bound certifies nothing). mstate: bit 0 the m-list
// is certified, bit 1 the best match is (the rule of k_sweep), bit 2 an owner
// (a non-flat window).
__global__ void k_mth_select(const double* __restrict__ A, const double* __restrict__ invn,
                             const double* __restrict__ sig, const uint8_t* __restrict__ flat,
                             const int32_t* __restrict__ hc, const double* __restrict__ hS,
                             const int32_t* __restrict__ hn, const double* __restrict__ hbound,
                             const double* __restrict__ hsig, const unsigned long long* __restrict__ rflat,
                             int fresh, int p, int m, int64_t N,
                             int64_t N0, int L, int64_t e, int base, double margin, double* __restrict__ vals,
                             int32_t* __restrict__ nn, double* __restrict__ ub, uint8_t* __restrict__ mstate,
                             unsigned long long* __restrict__ n_open) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = o < N;
  const bool owner = live && !flat[o];
  bool cert_m = false;
  if (owner) {
    const int nh = hn[o];
    const double Ao = A[o], io = invn[o];
    const double lb = unstored_bound(o, base, sig, hbound, hsig, fresh ? 0.0 : __longlong_as_double((long long)*rflat));
    const double twoL = 2.0 * (double)L;
    auto dist = [&](double u) { return sqrt(twoL * (u > 0.0 ? u : 0.0)); };
    auto below = [&](double d) { return lb == INFINITY || d < lb * (1.0 - 1.0e-12); };
    uint64_t prev = 0;
    int cnt = 0;
    bool cert_1 = false;
    for (int j = 0; j < m; ++j) {
      uint64_t kb = kEmptyKey;
      double rb = -2.0;
      for (int r = 0; r < nh; ++r) {
        const int64_t c = hc[o * p + r];
        if (c >= N || iabs64(c - o) <= e || flat[c]) continue;
        const double rho = rho_from_sum(hS[o * p + r], Ao, A[c], L, io, invn[c]);
        const uint64_t k = make_key(rho, c);
        if (j > 0 && k <= prev) continue;
        if (k < kb) {
          kb = k;
          rb = rho;
        }
      }
      if (kb == kEmptyKey) break;
      prev = kb;
      cnt = j + 1;
      vals[(int64_t)j * N0 + o] = dist(1.0 - rb);
      nn[(int64_t)j * N0 + o] = (int32_t)key_cand(kb);
      ub[(int64_t)j * N0 + o] = dist(1.0 - rb + 2.0 * margin);
      const bool ok = below(dist(1.0 - rb + margin));
      if (j == 0) cert_1 = ok;
      if (j == m - 1) cert_m = ok;
    }
    if (cnt < m) cert_m = lb == INFINITY;  // a complete profile: the owner has no more candidates
    for (int j = cnt; j < m; ++j) {
      vals[(int64_t)j * N0 + o] = INFINITY;
      nn[(int64_t)j * N0 + o] = -1;
      ub[(int64_t)j * N0 + o] = INFINITY;
    }
    if (!cert_m)
      for (int j = 0; j < cnt; ++j) {  // no entry until the owner is resolved
        vals[(int64_t)j * N0 + o] = INFINITY;
        nn[(int64_t)j * N0 + o] = -1;
      }
    mstate[o] = (uint8_t)(4 | (cert_m ? 1 : 0) | (cert_1 ? 2 : 0));
  } else if (live) {
    for (int j = 0; j < m; ++j) {
      vals[(int64_t)j * N0 + o] = INFINITY;
      nn[(int64_t)j * N0 + o] = -1;
    }
    mstate[o] = 0;
  }
  count_wave(owner && !cert_m, n_open);
}

// After the certified owners' rankings with twice the exclusion zone: tau_j is
// the distance of the k-th owner taken for column j. Those k owners are pairwise
// more than 2e apart, so any window excludes at most one of them, and the
// greedy ranking of all owners (exclusion e) takes k owners at distance >= tau_j
// whatever the unresolved owners turn out to be. An unresolved owner whose upper
// bounds lie below tau_j in every column is never examined before the k-th pick
// of any column: its m-list is left out (pruned). The others are listed for the
// top-m row recompute; with !best_exact, a pruned owner whose best match is not
// certified goes to the best-match recompute list.
__global__ void k_mth_prune(const uint8_t* __restrict__ mstate, const double* __restrict__ ub,
                            const double* __restrict__ tau_d, int64_t N, int64_t N0, int m, int kd, int best_exact,
                            int32_t* __restrict__ mlist, unsigned long long* __restrict__ nmlist,
                            int32_t* __restrict__ fail, unsigned long long* __restrict__ nfail,
                            unsigned long long* __restrict__ ncert, unsigned long long* __restrict__ npruned) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint8_t st = o < N ? mstate[o] : 0;
  const bool open = (st & 4) && !(st & 1);
  bool need = false;
  if (open) {
    for (int j = 0; j < m && !need; ++j) {
      const double t = tau_d[(int64_t)j * kd + kd - 1];
      need = !(t == t) || !(ub[(int64_t)j * N0 + o] * (1.0 + 1.0e-12) < t);
    }
  }
  count_wave((st & 4) && (st & 1), ncert);
  count_wave(open && !need, npruned);
  push_fail_wave(open && need, mlist, nmlist, o);
  push_fail_wave(open && !need && !best_exact && !(st & 2), fail, nfail, o);
}

// exact j-th best-match distances of the recomputed owners (direct FP64 sums)
__global__ void k_mth_fill(const double* __restrict__ xs, const double* __restrict__ A,
                           const double* __restrict__ invn, const int32_t* __restrict__ list,
                           const unsigned long long* __restrict__ nlist, const uint64_t* __restrict__ keys, int m,
                           int64_t N0, int L, double* __restrict__ vals, int32_t* __restrict__ nn) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= (int64_t)*nlist) return;
  const int64_t o = list[w];
  for (int j = 0; j < m; ++j) {
    const uint64_t k = keys[o * m + j];
    double d = INFINITY;
    int32_t c = -1;
    if (k != kEmptyKey) {
      c = (int32_t)key_cand(k);
      const double rho = rho_from_sum(cross_sum(xs, L, o, c), A[o], A[c], L, invn[o], invn[c]);
      const double u = 1.0 - rho;
      d = sqrt(2.0 * (double)L * (u > 0.0 ? u : 0.0));
    }
    vals[(int64_t)j * N0 + o] = d;
    nn[(int64_t)j * N0 + o] = c;
  }
}

// the best key of every recomputed owner (its first of m)
__global__ void k_topm_best(const int32_t* __restrict__ list, const unsigned long long* __restrict__ nlist, int m,
                            const uint64_t* __restrict__ keys, uint64_t* __restrict__ best) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= (int64_t)*nlist) return;
  const int64_t o = list[w];
  best[o] = keys[o * m];
}

hipError_t launch_mth_select(const MthSelect& a, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  if (a.m < 1 || a.m > a.p) return hipErrorInvalidValue;
  k_mth_select<<<blocks_for(a.N, 128), 128, 0, st>>>(a.A, a.invn, a.sig, a.flat, a.hc, a.hS, a.hn, a.hbound, a.hsig,
                                                     a.rflat, a.fresh, a.p, a.m, a.N,
                                                     a.N0, a.L, a.e, a.base, a.margin, a.vals, a.nn, a.ub, a.mstate,
                                                     a.n_open);
  return hipGetLastError();
}

hipError_t launch_mth_prune(const uint8_t* mstate, const double* ub, const double* tau_d, int64_t N, int64_t N0,
                            int m, int kd, int best_exact, int32_t* mlist, unsigned long long* nmlist, int32_t* fail,
                            unsigned long long* nfail, unsigned long long* ncert, unsigned long long* npruned,
                            hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_mth_prune<<<blocks_for(N, 256), 256, 0, st>>>(mstate, ub, tau_d, N, N0, m, kd, best_exact, mlist, nmlist, fail,
                                                  nfail, ncert, npruned);
  return hipGetLastError();
}

hipError_t launch_recompute_topm_keys(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                      const int32_t* list, const unsigned long long* nlist, int64_t max_listed,
                                      int64_t N, int64_t N0, int L, int64_t e, int m, uint64_t* keys, uint64_t* best,
                                      double* vals, int32_t* nn, bool mfma, hipStream_t st) {
  if (max_listed <= 0 || N <= 0) return hipSuccess;
  k_clear_keys<<<blocks_for(max_listed, 256), 256, 0, st>>>(list, nlist, m, keys);
  const dim3 grid(blocks_for(N, kWave * kRecK), (unsigned)(max_listed < 32 ? max_listed : 32));
  for (int j = 0; j < m; ++j) {
    if (mfma) {
      const hipError_t e1 = launch_recompute_round_mfma(xs, A, invn, flat, list, nlist, max_listed, N, L, e, m, j,
                                                        keys, st);
      if (e1 != hipSuccess) return e1;
    } else {
      k_recompute_round<<<grid, kWave, 0, st>>>(xs, A, invn, flat, list, nlist, N, L, e, m, j, keys);
    }
  }
  k_topm_best<<<blocks_for(max_listed, 256), 256, 0, st>>>(list, nlist, m, keys, best);
  k_mth_fill<<<blocks_for(max_listed, 128), 128, 0, st>>>(xs, A, invn, list, nlist, keys, m, N0, L, vals, nn);
  return hipGetLastError();
}

hipError_t launch_recompute_topm(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                 const int32_t* fail, const unsigned long long* nfail, int64_t max_listed, int64_t N,
                                 int L, int64_t e, int m, int p, uint64_t* keys, int32_t* hc, double* hS, int32_t* hn,
                                 uint64_t* best, bool mfma, hipStream_t st) {
  if (max_listed <= 0 || N <= 0) return hipSuccess;
  if (m < 1 || m > p) return hipErrorInvalidValue;
  k_clear_keys<<<blocks_for(max_listed, 256), 256, 0, st>>>(fail, nfail, m, keys);
  const dim3 grid(blocks_for(N, kWave * kRecK), (unsigned)(max_listed < 32 ? max_listed : 32));
  for (int j = 0; j < m; ++j) {
    if (mfma) {
      const hipError_t e1 = launch_recompute_round_mfma(xs, A, invn, flat, fail, nfail, max_listed, N, L, e, m, j,
                                                        keys, st);
      if (e1 != hipSuccess) return e1;
    } else {
      k_recompute_round<<<grid, kWave, 0, st>>>(xs, A, invn, flat, fail, nfail, N, L, e, m, j, keys);
    }
  }
  k_topm_store<<<blocks_for(max_listed, 256), 256, 0, st>>>(xs, fail, nfail, L, m, p, keys, hc, hS, hn, best);
  return hipGetLastError();
}

hipError_t launch_mth_values(const double* A, const double* invn, const uint8_t* flat, const int32_t* hc,
                             const double* hS, const int32_t* hn, int p, int m, int64_t N, int64_t N0, int L,
                             double* vals, int32_t* nn, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_mth_values<<<blocks_for(N, 256), 256, 0, st>>>(A, invn, flat, hc, hS, hn, p, m, N, N0, L, vals, nn);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Thresholds of a rebuild from the partial profiles it replaces. After the sweep
// at L, an owner whose profile holds p candidates all still eligible at L has p
// real candidates with correlations evaluated from their sums (error <= margin):
// the smallest of them, lowered by the margin, is at most the owner's true p-th
// largest correlation, so it is a valid threshold for the collecting pass with p
// thresholds, and on periodic series a far tighter one than the p-th best seed.
// thrp[o] = that value, or -inf when the profile cannot give one.
__global__ void k_profile_threshold(const double* __restrict__ A, const double* __restrict__ invn,
                                    const uint8_t* __restrict__ flat, const int32_t* __restrict__ hc,
                                    const double* __restrict__ hS, const int32_t* __restrict__ hn, int p, int64_t N,
                                    int L, int64_t e, double margin, double* __restrict__ thrp) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  double t = -INFINITY;
  if (!flat[o] && hn[o] == p) {
    const double Ao = A[o], io = invn[o];
    double lo = INFINITY;
    bool all = true;
    for (int r = 0; r < p && all; ++r) {
      const int64_t c = hc[o * p + r];
      all = c < N && iabs64(c - o) > e && !flat[c];
      if (all) lo = fmin(lo, rho_from_sum(hS[o * p + r], Ao, A[c], L, io, invn[c]));
    }
    if (all) t = lo - margin;
  }
  thrp[o] = t;
}

// the collecting thresholds raised to the profile thresholds (both are at most
// the true p-th largest correlation, so their maximum is as well); an owner that
// the seeding left without a threshold (no eligible seed) takes the profile's
__global__ void k_tighten_threshold(const double* __restrict__ thrp, int64_t N, double* __restrict__ thr,
                                    float* __restrict__ thr32) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  const double tp = thrp[o];
  if (!(tp > -INFINITY)) return;
  const double t = thr[o];
  if (t >= 2.0 || tp > t) {
    thr[o] = tp;
    if (thr32) thr32[o] = __double2float_rd(tp);
  }
}

hipError_t launch_profile_threshold(const double* A, const double* invn, const uint8_t* flat, const int32_t* hc,
                                    const double* hS, const int32_t* hn, int p, int64_t N, int L, int64_t e,
                                    double margin, double* thrp, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_profile_threshold<<<blocks_for(N, 256), 256, 0, st>>>(A, invn, flat, hc, hS, hn, p, N, L, e, margin, thrp);
  return hipGetLastError();
}

hipError_t launch_tighten_threshold(const double* thrp, int64_t N, double* thr, float* thr32, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_tighten_threshold<<<blocks_for(N, 256), 256, 0, st>>>(thrp, N, thr, thr32);
  return hipGetLastError();
}

hipError_t launch_seed_append(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                              const int32_t* src, int64_t N, int L, int64_t e, int p, int D, double margin,
                              int best_exact, double* thr, float* thr32, uint32_t* cnt, int32_t* fail,
                              unsigned long long* nfail, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (D < 0 || 4 * D + 2 > kWave) return hipErrorInvalidValue;
  const int seeds = 4 * D + 2;  // D = 0: the single candidate src[o], one lane per owner
#define SEED_LAUNCH(G)                                                                                     \
  k_seed_append<G><<<blocks_for(N, kWave / (G)), kWave, 0, st>>>(xs, A, invn, flat, src, N, L, e, p, D, margin, \
                                                                 best_exact, thr, thr32, cnt, fail, nfail)
  if (D == 0)
    SEED_LAUNCH(1);
  else if (seeds <= 8)
    SEED_LAUNCH(8);
  else if (seeds <= 16)
    SEED_LAUNCH(16);
  else if (seeds <= 32)
    SEED_LAUNCH(32);
  else
    SEED_LAUNCH(64);
#undef SEED_LAUNCH
  return hipGetLastError();
}

hipError_t launch_merge(const double* xs, const double* A, const double* invn, const double* sig, const uint8_t* flat,
                        const double* thr, const uint32_t* cnt, const int32_t* buf, int64_t cap, int64_t N, int L,
                        int p, int keep, double margin, int best_exact, int32_t* hc, double* hS, int32_t* hn,
                        double* hbound, double* hsig, uint8_t* hflat, uint64_t* best, int32_t* fail,
                        unsigned long long* nfail, int32_t* big, unsigned long long* nbig, unsigned long long* nappend,
                        unsigned long long* nover, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (cap <= 0 || cap > kMergeCap || keep < 0 || keep > p) return hipErrorInvalidValue;
  k_merge_small<<<blocks_for(N, kWave / kSmallG), kWave, 0, st>>>(xs, A, invn, sig, flat, thr, cnt, buf, cap, N, L, p,
                                                                   keep, margin, best_exact, hc, hS, hn, hbound, hsig,
                                                                   hflat, best, fail, nfail, big, nbig, nover);
  // a wavefront per listed owner; 4,096 workgroups fill the chip (the list is
  // walked in a grid-stride loop, so a short list costs little to dispatch)
  k_merge_big<<<(unsigned)(N < 4096 ? N : 4096), kWave, (size_t)cap * 3 * sizeof(double), st>>>(
      xs, A, invn, sig, thr, cnt, buf, cap, N, L, p, keep, margin, hc, hS, hn, hbound, hsig, best, big, nbig);
  k_sum_counts<<<64, 1024, 0, st>>>(cnt, N, nappend);
  return hipGetLastError();
}

hipError_t launch_sweep(const double* xs, const double* A, const double* invn, const double* sig, const uint8_t* flat,
                        int64_t N, int L, int64_t e, int p, int base, const int32_t* hc, double* hS, const int32_t* hn,
                        const double* hbound, const double* hsig, const unsigned long long* rflat, double margin,
                        uint64_t* best, int32_t* fail, unsigned long long* nfail, unsigned long long* nvalid,
                        double* lbm, unsigned long long* min_dist, unsigned long long* min_lb, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (!rflat) return hipErrorInvalidValue;
  k_sweep<<<blocks_for(N, 128), 128, 0, st>>>(xs, A, invn, sig, flat, N, L, e, p, base, hc, hS, hn, hbound, hsig,
                                               rflat, margin, best, fail, nfail, nvalid, lbm, min_dist, min_lb);
  return hipGetLastError();
}

hipError_t launch_split_fail(const int32_t* fail, const unsigned long long* nfail, int64_t max_listed,
                             const double* lbm, const unsigned long long* limit, int all_partial, int32_t* rec,
                             unsigned long long* nrec, int32_t* part, unsigned long long* npart, hipStream_t st) {
  if (max_listed <= 0) return hipSuccess;
  k_split_fail<<<blocks_for(max_listed, 256), 256, 0, st>>>(fail, nfail, lbm, limit, all_partial, rec, nrec, part,
                                                             npart);
  return hipGetLastError();
}

hipError_t launch_mark_partial(const int32_t* part, const unsigned long long* npart, int64_t max_listed,
                               const double* lbm, double* prof_dist, int32_t* prof_idx, hipStream_t st) {
  if (max_listed <= 0) return hipSuccess;
  k_mark_partial<<<blocks_for(max_listed, 256), 256, 0, st>>>(part, npart, lbm, prof_dist, prof_idx);
  return hipGetLastError();
}

hipError_t launch_recompute(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                            const int32_t* fail, const unsigned long long* nfail, int64_t max_listed, int64_t N,
                            int L, int64_t e, uint64_t* best, hipStream_t st) {
  if (max_listed <= 0 || N <= 0) return hipSuccess;
  const dim3 grid(blocks_for(N, kWave * kRecK), (unsigned)(max_listed < 32 ? max_listed : 32));
  k_recompute<<<grid, kWave, 0, st>>>(xs, A, invn, flat, fail, nfail, N, L, e, best);
  return hipGetLastError();
}

}  // namespace valmod
