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
// at least sqrt(b (1 - max(bound_rho, 0)^2)) sigma_{o,b} / sigma_{o,L}.
#include "valmod_common.h"
#include "valmod_kernels.h"

#include <math.h>

namespace valmod {

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// anchored cross sum of windows o and c at length L (direct, L - 1 FMAs)
__device__ __forceinline__ double cross_sum(const double* __restrict__ xs, int L, int64_t o, int64_t c) {
  const double xo = xs[o], xc = xs[c];
  double s = 0.0;
  for (int k = 1; k < L; ++k) s = fma(xs[o + k] - xo, xs[c + k] - xc, s);
  return s;
}

__device__ __forceinline__ double rho_from_sum(double S, double Ao, double Ac, int L, double io, double ic) {
  return (S - Ao * Ac / (double)L) * io * ic;
}

__device__ __forceinline__ void push_fail(int32_t* fail, unsigned long long* nfail, int64_t o) {
  const unsigned long long pos = atomicAdd(nfail, 1ull);
  fail[pos] = (int32_t)o;
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
// recompute list. One wavefront per owner.
__global__ __launch_bounds__(kWave) void k_seed_append(const double* __restrict__ xs, const double* __restrict__ A,
                                                       const double* __restrict__ invn,
                                                       const uint8_t* __restrict__ flat,
                                                       const int32_t* __restrict__ src, int64_t N, int L, int64_t e,
                                                       int p, int D, double margin, int best_exact,
                                                       double* __restrict__ thr,
                                                       uint32_t* __restrict__ cnt, int32_t* __restrict__ fail,
                                                       unsigned long long* __restrict__ nfail) {
  const int64_t o = blockIdx.x;
  const int t = threadIdx.x;
  if (o >= N) return;
  if (t == 0) cnt[o] = 0;
  if (flat[o]) {
    if (t == 0) thr[o] = 3.0;  // not an owner
    return;
  }
  int64_t c = -1;
  if (t <= 2 * D) {
    const int64_t d = t - D, w = o + d;
    if (w >= 0 && w < N && src[w] >= 0) c = (int64_t)src[w] - d;
  } else if (t <= 4 * D + 1) {
    const int64_t d = t - (3 * D + 1);
    if (src[o] >= 0) c = (int64_t)src[o] + d;
  }
  bool ok = c >= 0 && c < N && iabs64(c - o) > e && !flat[c];
  // drop duplicates: keep the lowest lane holding each candidate
  for (int m = 0; m < kWave; ++m) {
    const int64_t oc = (int64_t)__shfl((int)c, m, kWave);
    const int ov = __shfl((int)ok, m, kWave);
    if (m < t && ov && oc == c) ok = false;
  }
  uint64_t key = kEmptyKey;
  double rho = -2.0;
  if (ok) {
    rho = rho_from_sum(cross_sum(xs, L, o, c), A[o], A[c], L, invn[o], invn[c]);
    key = make_key(rho, c);
  }
  const int m = __popcll(__ballot(ok));
  const int rank = wave_rank(key, ok);
  if (m == 0) {
    if (t == 0) {
      thr[o] = 3.0;
      if (!best_exact) push_fail(fail, nfail, o);
    }
    return;
  }
  if ((int64_t)p >= N - 1) {
    if (t == 0) thr[o] = -2.0 - margin;  // a profile can hold every candidate: collect them all
    return;
  }
  const int want = (p < m ? p : m) - 1;
  if (ok && rank == want) thr[o] = rho - margin;
}

// --------------------------------------------------------------------------
// Merge of the collected candidates into the partial profile of each owner at
// the new base length L: exact correlation of every candidate the pass
// appended, top-p by (correlation desc, index asc), the bound correlation of
// the ones not kept, and the owner's best key. Owners whose list overflowed
// (incomplete) or that collected nothing go to the recompute list with an empty
// profile. One wavefront per owner.
constexpr int kMergeCap = 512;

__global__ __launch_bounds__(kWave) void k_merge(
    const double* __restrict__ xs, const double* __restrict__ A, const double* __restrict__ invn,
    const double* __restrict__ sig, const uint8_t* __restrict__ flat, const double* __restrict__ thr,
    const uint32_t* __restrict__ cnt, const int32_t* __restrict__ buf, int64_t cap, int64_t N, int L, int p,
    int keep, double margin, int best_exact, int32_t* __restrict__ hc, double* __restrict__ hS, int32_t* __restrict__ hn,
    double* __restrict__ hbound, double* __restrict__ hsig, uint64_t* __restrict__ best, int32_t* __restrict__ fail,
    unsigned long long* __restrict__ nfail, unsigned long long* __restrict__ nappend) {
  // best_exact: `best` already holds every owner's exact neighbour (a
  // matrix-profile pass ran at this length), so an owner whose profile cannot be
  // built keeps it instead of going to the recompute list.
  __shared__ uint64_t skey[kMergeCap];
  __shared__ double srho[kMergeCap];
  __shared__ double ssum[kMergeCap];
  __shared__ double sbound;
  const int64_t o = blockIdx.x;
  const int t = threadIdx.x;
  if (o >= N) return;
  const uint32_t total = cnt[o];
  if (t == 0 && total) atomicAdd(nappend, (unsigned long long)total);
  if (flat[o] || thr[o] >= 2.0) {  // not an owner, or already queued for recompute by the seeding
    if (t == 0) {
      hn[o] = 0;
      if (!best_exact || flat[o]) best[o] = kEmptyKey;
    }
    return;
  }
  const int64_t m = total;
  if (m == 0 || m > cap || m > kMergeCap) {
    if (t == 0) {
      hn[o] = 0;
      if (!best_exact) {
        best[o] = kEmptyKey;
        push_fail(fail, nfail, o);
      }
    }
    return;
  }
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
  // every candidate not collected is below the threshold (up to the pass rounding);
  // below -1 every candidate was collected, and -3 marks a complete profile
  if (t == 0) sbound = thr[o] < -1.5 ? -3.0 : thr[o] + 2.0 * margin;
  __syncthreads();
  for (int64_t r = t; r < m; r += kWave) {
    const uint64_t k = skey[r];
    int64_t rank = 0;
    for (int64_t s2 = 0; s2 < m; ++s2) rank += skey[s2] < k ? 1 : 0;
    if (rank < keep) {
      hc[o * p + rank] = (int32_t)key_cand(k);
      hS[o * p + rank] = ssum[r];
    }
    if (rank == 0) best[o] = k;
    if (rank == keep && srho[r] > sbound) sbound = srho[r];  // the best collected candidate not kept
  }
  __syncthreads();
  if (t == 0) {
    hn[o] = (int32_t)(m < keep ? m : keep);
    hbound[o] = sbound;
    hsig[o] = sig[o];
  }
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
                        const double* __restrict__ hsig, uint64_t* __restrict__ best, int32_t* __restrict__ fail,
                        unsigned long long* __restrict__ nfail, unsigned long long* __restrict__ nvalid) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  if (flat[o]) {
    best[o] = kEmptyKey;
    return;
  }
  const int nh = hn[o];
  const double xo = xs[o], dx = xs[o + L - 1] - xo;
  const double Ao = A[o], io = invn[o];
  uint64_t kb = kEmptyKey;
  double rb = -2.0;
  for (int r = 0; r < nh; ++r) {
    const int64_t c = hc[o * p + r];
    if (c >= N) continue;  // no window of length L at c (nor at any longer length)
    const double S = fma(dx, xs[c + L - 1] - xs[c], hS[o * p + r]);
    hS[o * p + r] = S;
    if (iabs64(c - o) <= e || flat[c]) continue;
    const double rho = rho_from_sum(S, Ao, A[c], L, io, invn[c]);
    const uint64_t k = make_key(rho, c);
    if (k < kb) {
      kb = k;
      rb = rho;
    }
  }
  bool valid = false;
  if (kb != kEmptyKey && hsig[o] > 0.0) {
    const double u = 1.0 - rb;
    const double min_dist = sqrt(2.0 * (double)L * (u > 0.0 ? u : 0.0));
    if (hbound[o] < -2.5) {
      valid = true;  // complete profile: no candidate was left out
    } else {
      const double q = hbound[o] > 0.0 ? (hbound[o] < 1.0 ? hbound[o] : 1.0) : 0.0;
      const double max_lb = sqrt((double)base * (1.0 - q * q)) * hsig[o] / sig[o];
      valid = min_dist < max_lb * (1.0 - 1.0e-9);
    }
  }
  if (valid) {
    best[o] = kb;
    atomicAdd(nvalid, 1ull);
  } else {
    best[o] = kEmptyKey;
    push_fail(fail, nfail, o);
  }
}

// --------------------------------------------------------------------------
// Exact row recompute of the listed owners: the whole distance profile at L
// (every eligible candidate, anchored cross sums formed directly), reduced to
// the best key. One wavefront per listed owner.
__global__ __launch_bounds__(kWave) void k_recompute(const double* __restrict__ xs, const double* __restrict__ A,
                                                     const double* __restrict__ invn,
                                                     const uint8_t* __restrict__ flat,
                                                     const int32_t* __restrict__ fail, int64_t nfail, int64_t N,
                                                     int L, int64_t e, uint64_t* __restrict__ best) {
  const int64_t w = blockIdx.x;
  if (w >= nfail) return;
  const int t = threadIdx.x;
  const int64_t o = fail[w];
  const double Ao = A[o], io = invn[o];
  uint64_t kb = kEmptyKey;
  if (!flat[o]) {
    for (int64_t c = t; c < N; c += kWave) {
      if (iabs64(c - o) <= e || flat[c]) continue;
      const double rho = rho_from_sum(cross_sum(xs, L, o, c), Ao, A[c], L, io, invn[c]);
      const uint64_t k = make_key(rho, c);
      kb = k < kb ? k : kb;
    }
  }
  kb = wave_min_u64(kb);
  if (t == 0) best[o] = kb;
}

hipError_t launch_seed_append(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                              const int32_t* src, int64_t N, int L, int64_t e, int p, int D, double margin,
                              int best_exact, double* thr, uint32_t* cnt, int32_t* fail, unsigned long long* nfail,
                              hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_seed_append<<<(unsigned)N, kWave, 0, st>>>(xs, A, invn, flat, src, N, L, e, p, D, margin, best_exact, thr, cnt,
                                               fail, nfail);
  return hipGetLastError();
}

hipError_t launch_merge(const double* xs, const double* A, const double* invn, const double* sig, const uint8_t* flat,
                        const double* thr, const uint32_t* cnt, const int32_t* buf, int64_t cap, int64_t N, int L,
                        int p, int keep, double margin, int best_exact, int32_t* hc, double* hS, int32_t* hn,
                        double* hbound, double* hsig, uint64_t* best, int32_t* fail, unsigned long long* nfail,
                        unsigned long long* nappend, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_merge<<<(unsigned)N, kWave, 0, st>>>(xs, A, invn, sig, flat, thr, cnt, buf, cap, N, L, p, keep, margin,
                                        best_exact, hc, hS, hn, hbound, hsig, best, fail, nfail, nappend);
  return hipGetLastError();
}

hipError_t launch_sweep(const double* xs, const double* A, const double* invn, const double* sig, const uint8_t* flat,
                        int64_t N, int L, int64_t e, int p, int base, const int32_t* hc, double* hS, const int32_t* hn,
                        const double* hbound, const double* hsig, uint64_t* best, int32_t* fail,
                        unsigned long long* nfail, unsigned long long* nvalid, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_sweep<<<blocks_for(N, 128), 128, 0, st>>>(xs, A, invn, sig, flat, N, L, e, p, base, hc, hS, hn, hbound, hsig,
                                               best, fail, nfail, nvalid);
  return hipGetLastError();
}

hipError_t launch_recompute(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                            const int32_t* fail, int64_t nfail, int64_t N, int L, int64_t e, uint64_t* best,
                            hipStream_t st) {
  if (nfail <= 0) return hipSuccess;
  k_recompute<<<(unsigned)nfail, kWave, 0, st>>>(xs, A, invn, flat, fail, nfail, N, L, e, best);
  return hipGetLastError();
}

}  // namespace valmod
