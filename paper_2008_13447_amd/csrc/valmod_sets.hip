// Variable-length motif sets (Def. data series motif set; Problem of
// variable-length motif sets discovery; Sec. "Finding Motif Sets").
//
// For each of the top-k motif pairs (a, b, L, d) of a series, in rank order, the
// set holds the windows of length L whose distance to a or to b is below
// r = D * d, taken in order of (distance to the nearer member, offset); a window
// is skipped if it is a trivial match of a window already in the set or if an
// earlier set already holds its offset (the sets are disjoint by offset).
//
// The GPU computes every candidate's distance directly (the distance profile
// of both members in range), which is what the paper's recompute branch does;
// the branch that filters a kept partial profile returns the same windows. The
// steps are
//   1. k_set_centers    statistics of the 2k members, radius of each set;
//   2. k_set_candidates one lane per (set, window): statistics of the window,
//                       z-normalised distances to both members, append of the
//                       windows inside the radius with a sort key;
//   3. a stable LSD radix sort of the keys (set, distance, offset), 8 passes of
//      8 bits (k_rs_hist, k_rs_scan, k_rs_scatter);
//   4. k_set_greedy     one workgroup walks the sorted candidates in chunks of
//                       8192 and takes the members; conflicts inside a chunk
//                       are resolved by one wavefront, lane by lane with ballots.
// Every launch reads the candidate count on the device, so the sequence takes
// no host decision.
#include "valmod_common.h"
#include "valmod_kernels.h"

#include <math.h>

#include <stdlib.h>

#include <algorithm>
#include <utility>

namespace valmod {

namespace {

constexpr int kSetBits = 6;                // set index bits of a sort key (k <= 64)
constexpr int kQBits = 64 - kSetBits - kIdxBits;  // 36 bits of quantised distance
constexpr int kRsTile = 4096;              // radix-sort elements per tile
constexpr int kRsBins = 256;

// window statistics with the arithmetic of the per-length statistics kernel
// (anchored sums over k = 1..L-1), so flat decisions agree with the profile
__device__ __forceinline__ void window_stats(const double* __restrict__ xs, int64_t c, int L, double flat_eps,
                                             double& mu, double& inv, bool& flat) {
  const double x0 = xs[c];
  double a = 0.0, b = 0.0;
  for (int k = 1; k < L; ++k) {
    const double d = xs[c + k] - x0;
    a += d;
    b = fma(d, d, b);
  }
  const double m = a / (double)L;
  double v = b / (double)L - m * m;
  v = v > 0.0 ? v : 0.0;
  const double s = sqrt(v);
  mu = x0 + m;
  flat = s <= flat_eps * fmax(1.0, fabs(mu));
  inv = flat ? 0.0 : 1.0 / s;
}

// meta layout (doubles): [0, 2k) member means, [2k, 4k) member 1/sigma (0: flat), [4k, 5k) radius
// A rank without a pair (or with a pair outside the series) gets radius 0 and no candidates.
__global__ __launch_bounds__(kWave) void k_set_centers(const double* __restrict__ xs, int64_t n,
                                                       const int32_t* __restrict__ abl, const double* __restrict__ gd,
                                                       int k, double D, double flat_eps, double* __restrict__ meta) {
  const int t = threadIdx.x;
  if (t >= 2 * k) return;
  const int s = t >> 1;
  const int64_t a = abl[3 * s], b = abl[3 * s + 1], L = abl[3 * s + 2];
  const bool ok = a >= 0 && b >= 0 && L >= 2 && a + L <= n && b + L <= n;
  double mu = 0.0, inv = 0.0;
  bool flat = true;
  if (ok) window_stats(xs, (t & 1) ? b : a, (int)L, flat_eps, mu, inv, flat);
  meta[t] = mu;
  meta[2 * k + t] = flat ? 0.0 : inv;
  if ((t & 1) == 0) meta[4 * k + s] = ok ? D * gd[2 * s] : 0.0;
}

__global__ __launch_bounds__(256) void k_set_candidates(const double* __restrict__ xs, int64_t n,
                                                        const int32_t* __restrict__ abl, int k, double flat_eps,
                                                        const double* __restrict__ meta,
                                                        uint32_t* __restrict__ count, uint64_t* __restrict__ keys,
                                                        double* __restrict__ vals) {
  const int s = blockIdx.y;
  const int32_t a = abl[3 * s], b = abl[3 * s + 1];
  const int L = abl[3 * s + 2];
  const double r = meta[4 * k + s];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t NL = n - (int64_t)L + 1;
  bool member = false;
  double near = INFINITY;
  if (r > 0.0 && c < NL) {  // r > 0 only for a pair inside the series
    double mu, ic;
    bool flat;
    window_stats(xs, c, L, flat_eps, mu, ic, flat);
    const double ma = meta[2 * s], mb = meta[2 * s + 1];
    const double ia = meta[2 * k + 2 * s], ib = meta[2 * k + 2 * s + 1];
    if (!flat && (ia > 0.0 || ib > 0.0)) {
      // z-normalised differences (Eq. 6 by direct differences), both members at once
      double acc_a = 0.0, acc_b = 0.0;
      for (int q = 0; q < L; ++q) {
        const double zc = (xs[c + q] - mu) * ic;
        const double za = (xs[a + q] - ma) * ia - zc;
        const double zb = (xs[b + q] - mb) * ib - zc;
        acc_a = fma(za, za, acc_a);
        acc_b = fma(zb, zb, acc_b);
      }
      const double da = ia > 0.0 ? sqrt(acc_a) : INFINITY;
      const double db = ib > 0.0 ? sqrt(acc_b) : INFINITY;
      near = da < db ? da : db;
      member = near < r;
    }
  }
  // wavefront-aggregated append
  const uint64_t bal = __ballot(member);
  if (bal == 0) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)bal) - 1;
  uint32_t base = 0;
  if (lane == leader) {
    base = atomicAdd(count, (uint32_t)__popcll(bal));
    atomicAdd(count + 1 + s, (uint32_t)__popcll(bal));
  }
  base = (uint32_t)__shfl((int)base, leader, kWave);
  if (member) {
    const uint32_t rank = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
    double f = near / r * (double)(1ull << kQBits);
    uint64_t q = f < (double)((1ull << kQBits) - 1) ? (uint64_t)f : (1ull << kQBits) - 1;
    keys[base + rank] = ((uint64_t)s << (64 - kSetBits)) | (q << kIdxBits) | (uint64_t)c;
    vals[base + rank] = near;
  }
}

// --- stable LSD radix sort of (key, value) pairs, 8 bits per pass ---------
// hist[d * nb + tile]: count of digit d in tile (nb = tiles in use)
__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ count,
                                                 int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRsBins];
  const uint32_t M = *count;
  const uint32_t nb = (M + kRsTile - 1) / kRsTile;
  if (blockIdx.x >= nb) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t0 = blockIdx.x * kRsTile;
  for (uint32_t i = t0 + threadIdx.x; i < t0 + kRsTile && i < M; i += 256)
    atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// exclusive prefix over the digit-major histogram (one workgroup)
__global__ __launch_bounds__(1024) void k_rs_scan(const uint32_t* __restrict__ count, uint32_t* __restrict__ hist) {
  __shared__ uint32_t part[1024];
  const uint32_t M = *count;
  const uint32_t nb = (M + kRsTile - 1) / kRsTile;
  const uint32_t total = nb * kRsBins;
  const uint32_t per = (total + 1023) / 1024;
  const uint32_t lo = threadIdx.x * per;
  const uint32_t hi = lo + per < total ? lo + per : total;
  uint32_t sum = 0;
  for (uint32_t i = lo; i < hi; ++i) sum += hist[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 1024 partial sums
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = threadIdx.x >= (uint32_t)o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = hist[i];
    hist[i] = run;
    run += v;
  }
}

// one wavefront per tile, elements in tile order; equal digits keep their order
__global__ __launch_bounds__(kWave) void k_rs_scatter(const uint64_t* __restrict__ kin, const double* __restrict__ vin,
                                                      const uint32_t* __restrict__ count, int shift,
                                                      const uint32_t* __restrict__ hist, uint64_t* __restrict__ kout,
                                                      double* __restrict__ vout) {
  __shared__ uint32_t off[kRsBins];
  const uint32_t M = *count;
  const uint32_t nb = (M + kRsTile - 1) / kRsTile;
  if (blockIdx.x >= nb) return;
  const int lane = threadIdx.x;
  for (int d = lane; d < kRsBins; d += kWave) off[d] = hist[(size_t)d * nb + blockIdx.x];
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t t0 = blockIdx.x * kRsTile;
  for (int r = 0; r < kRsTile / kWave; ++r) {
    const uint32_t i = t0 + (uint32_t)(r * kWave + lane);
    const bool valid = i < M;
    uint64_t key = 0;
    double val = 0.0;
    if (valid) {
      key = kin[i];
      val = vin[i];
    }
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    if (peers == 0) break;
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bb = __ballot(valid && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & below);
    const uint32_t pos = off[d] + rank;
    __syncthreads();
    if (valid && rank == 0) off[d] += (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      kout[pos] = key;
      vout[pos] = val;
    }
  }
}

// --- greedy selection ------------------------------------------------------
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Clears the outputs, the taken-offset bitmap, the member buckets and the count.
__global__ __launch_bounds__(256) void k_set_init(int k, int64_t cap, int32_t* __restrict__ out_count,
                                                  int32_t* __restrict__ out_off, double* __restrict__ out_dist,
                                                  uint64_t* __restrict__ taken, int64_t nwords,
                                                  uint32_t* __restrict__ bucket, int64_t nbucket,
                                                  uint32_t* __restrict__ count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < (int64_t)k * cap; i += stride) {
    if (out_off) out_off[i] = -1;
    if (out_dist) out_dist[i] = NAN;
  }
  for (int64_t i = t0; i < k; i += stride) out_count[i] = 0;
  for (int64_t i = t0; i < nwords; i += stride) taken[i] = 0;
  for (int64_t i = t0; i < nbucket; i += stride) bucket[i] = 0;
  for (int64_t i = t0; i <= k; i += stride) count[i] = 0;
}

// bucket[c / (e + 1)] holds the member of the current set in that bucket as
// ((set + 1) << 22) | offset; members of one set are more than e apart, so a
// bucket of width e + 1 holds at most one, and a window conflicts with a
// member only if that member sits in its bucket or a neighbouring one.
// ATOMIC: loads that see stores of other lanes made since the last fence.
// (offsets are below 2^22, so 32-bit arithmetic is exact)
// The three loads are issued unconditionally (indices clamped into the map) so
// that they overlap.
template <bool ATOMIC>
__device__ __forceinline__ bool conflicts(const uint32_t* bucket, uint32_t nbucket, uint32_t c, uint32_t tag,
                                          uint32_t e) {
  const uint32_t bk = c / (e + 1);
  const uint32_t q0 = bk > 0 ? bk - 1 : 0, q2 = bk + 1 < nbucket ? bk + 1 : nbucket - 1;
  uint32_t v[3];
  if (ATOMIC) {
    v[0] = ld_u32(bucket + q0);
    v[1] = ld_u32(bucket + bk);
    v[2] = ld_u32(bucket + q2);
  } else {
    v[0] = bucket[q0];
    v[1] = bucket[bk];
    v[2] = bucket[q2];
  }
  bool hit = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const uint32_t m = v[d] & (uint32_t)kIdxMask;
    if ((v[d] >> kIdxBits) == tag && (c > m ? c - m : m - c) <= e) hit = true;
  }
  return hit;
}

__device__ __forceinline__ int readlane_i32(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

constexpr int kGreedyThreads = 1024;
constexpr int kGreedyPer = 8;                                // candidates per thread and chunk
constexpr int kGreedyChunk = kGreedyThreads * kGreedyPer;   // 8192
constexpr int kGreedySubs = kGreedyChunk / kWave;           // 128 groups of 64
constexpr int kLdsBuckets = 16384;                          // member buckets kept in LDS when they fit

// One workgroup walks the sets in rank order and each set's sorted candidates
// in chunks of 8192: all waves test the chunk against the members taken so far
// and the offsets of earlier sets and record, per group of 64, which candidates
// survive; wave 0 then settles the surviving groups in key order, testing each
// again against the members taken so far (including those of earlier groups
// of the chunk) and entering each new member in the bucket map; finally all
// waves write the new members out and mark their offsets as taken. The bucket map of a set lives
// in LDS when its n0 / (e + 1) + 2 buckets fit, else in the global array. The
// keys of the next chunk are loaded while the current one is settled.
__global__ __launch_bounds__(kGreedyThreads) void k_set_greedy(
    const uint64_t* __restrict__ keys, const double* __restrict__ vals, const uint32_t* __restrict__ count,
    const int32_t* __restrict__ abl, int excl_den, int k, int64_t cap, int64_t n0, int64_t lds_max,
    uint64_t* __restrict__ taken, uint32_t* __restrict__ bucket, int32_t* __restrict__ out_count,
    int32_t* __restrict__ out_off, double* __restrict__ out_dist) {
  __shared__ int32_t s_c[kGreedyChunk];
  __shared__ int32_t s_acc[kGreedyChunk];
  __shared__ uint64_t s_mask[kGreedySubs];
  __shared__ uint32_t s_bucket[kLdsBuckets];
  __shared__ int s_nacc;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const bool wave0 = tid < kWave;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int i = tid; i < kLdsBuckets; i += kGreedyThreads) s_bucket[i] = 0;  // tag 0: empty
  __syncthreads();
  // key of candidate u * 1024 + tid of the chunk starting at `at`
  auto load_keys = [&](uint32_t at, uint32_t end, uint64_t* kk) {
#pragma unroll
    for (int u = 0; u < kGreedyPer; ++u) {
      const uint32_t i = at + (uint32_t)(u * kGreedyThreads + tid);
      kk[u] = i < end ? keys[i] : 0;
    }
  };
  uint32_t start = 0;
  for (int s = 0; s < k; ++s) {
    const uint32_t len = count[1 + s];
    const uint32_t end = start + len;
    const uint32_t e = len ? (uint32_t)excl_zone(abl[3 * s + 2], excl_den) : 1u;
    const uint32_t nbk = (uint32_t)(n0 / (e + 1) + 2);
    const bool lds = (int64_t)nbk <= lds_max;
    const uint32_t tag = (uint32_t)(s + 1);
    int64_t got = 0;
    uint64_t kk[kGreedyPer];
    load_keys(start, end, kk);
    for (uint32_t base = start; base < end; base += kGreedyChunk) {
      const uint32_t cl = end - base < (uint32_t)kGreedyChunk ? end - base : (uint32_t)kGreedyChunk;
      // the fence that ended the previous chunk makes plain loads see its members and offsets
      // all taken-bitmap loads first (a key beyond the chunk is 0: offset 0, ignored)
      uint64_t tw[kGreedyPer];
#pragma unroll
      for (int u = 0; u < kGreedyPer; ++u) {
        const uint32_t c = (uint32_t)(kk[u] & kIdxMask);
        tw[u] = taken[c >> 6];
      }
#pragma unroll
      for (int u = 0; u < kGreedyPer; ++u) {
        const uint32_t j = (uint32_t)(u * kGreedyThreads + tid);
        const uint32_t c = (uint32_t)(kk[u] & kIdxMask);
        bool alive = false;
        if (j < cl) {
          s_c[j] = (int32_t)c;
          alive = !((tw[u] >> (c & 63)) & 1ull) && !(lds ? conflicts<false>(s_bucket, nbk, c, tag, e)
                                                         : conflicts<false>(bucket, nbk, c, tag, e));
        }
        const uint64_t bal = __ballot(alive);
        if (lane == 0) s_mask[u * (kGreedyThreads / kWave) + wave] = bal;
      }
      __syncthreads();
      // prefetch the next chunk of this set (the loads overlap the settling below)
      if (base + kGreedyChunk < end) load_keys(base + kGreedyChunk, end, kk);
      if (wave0) {
        int nacc = 0;
        for (int half = 0; half < kGreedySubs / kWave; ++half) {
          const uint64_t mine = s_mask[half * kWave + lane];
          uint64_t nz = __ballot(mine != 0);
          while (nz) {
            const int q = __ffsll((unsigned long long)nz) - 1;
            nz &= nz - 1;
            const uint64_t live = readlane_u64(mine, q);
            const uint32_t j = (uint32_t)((half * kWave + q) * kWave + lane);
            bool alive = (live >> lane) & 1ull;
            const uint32_t c = alive ? (uint32_t)s_c[j] : 0u;
            if (alive && (lds ? conflicts<false>(s_bucket, nbk, c, tag, e) : conflicts<true>(bucket, nbk, c, tag, e)))
              alive = false;
            uint64_t acc = 0;
            uint64_t am = __ballot(alive);
            while (am) {
              const int j0 = __ffsll((unsigned long long)am) - 1;
              const uint32_t cj = (uint32_t)readlane_i32((int)c, j0);
              acc |= 1ull << j0;
              if (lane == j0 || (alive && lane > j0 && (c > cj ? c - cj : cj - c) <= e)) alive = false;
              am = __ballot(alive);
            }
            if ((acc >> lane) & 1ull) {
              s_acc[nacc + __popcll(acc & below)] = (int32_t)j;  // written out below by all waves
              const uint32_t v = (tag << kIdxBits) | (uint32_t)c;
              if (lds)
                s_bucket[c / (e + 1)] = v;
              else
                __hip_atomic_store(bucket + c / (e + 1), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (acc && !lds) __threadfence_block();  // the next group reads the new members
            nacc += __popcll(acc);
          }
        }
        if (lane == 0) s_nacc = nacc;
      }
      __syncthreads();
      const int nacc = s_nacc;
      for (int t = tid; t < nacc; t += kGreedyThreads) {
        const int32_t j = s_acc[t];
        const int64_t c = s_c[j];
        const int64_t pos = got + t;
        if (pos < cap) {
          if (out_off) out_off[(int64_t)s * cap + pos] = (int32_t)c;
          if (out_dist) out_dist[(int64_t)s * cap + pos] = vals[base + (uint32_t)j];
        }
        __hip_atomic_fetch_or(taken + (c >> 6), 1ull << (c & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      got += nacc;
      __threadfence();
      __syncthreads();
    }
    if (tid == 0) out_count[s] = (int32_t)got;
    start = end;
  }
}

}  // namespace

size_t motif_sets_hist_words(int64_t cand_cap) {
  return (size_t)kRsBins * (size_t)((cand_cap + kRsTile - 1) / kRsTile + 1);
}

hipError_t launch_motif_sets(const MotifSetLaunch& m, hipStream_t st) {
  if (m.k < 1 || m.k > (1 << kSetBits) || m.cap < 1) return hipErrorInvalidValue;
  const int64_t nwords = (m.n0 + 63) / 64;
  const int64_t nbucket = m.n0 / 2 + 2;  // bucket width e + 1 >= 2
  const int64_t init_items = std::max<int64_t>(std::max<int64_t>((int64_t)m.k * m.cap, nwords), nbucket);
  const int64_t init_blocks = std::min<int64_t>((init_items + 255) / 256, 4096);
  k_set_init<<<dim3((unsigned)std::max<int64_t>(init_blocks, 1)), dim3(256), 0, st>>>(
      m.k, m.cap, m.out_count, m.out_off, m.out_dist, m.taken, nwords, m.bucket, nbucket, m.count);
  k_set_centers<<<dim3(1), dim3(kWave), 0, st>>>(m.xs, m.n, m.abl, m.gd, m.k, m.D, m.flat_eps, m.meta);
  // every set's length is at least the smallest one, so n0 windows bound each set
  k_set_candidates<<<dim3((unsigned)((m.n0 + 255) / 256), (unsigned)m.k), dim3(256), 0, st>>>(
      m.xs, m.n, m.abl, m.k, m.flat_eps, m.meta, m.count, m.keys0, m.vals0);
  const unsigned tiles = (unsigned)((m.cand_cap + kRsTile - 1) / kRsTile);
  uint64_t* kin = m.keys0;
  double* vin = m.vals0;
  uint64_t* kout = m.keys1;
  double* vout = m.vals1;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    k_rs_hist<<<dim3(tiles), dim3(256), 0, st>>>(kin, m.count, shift, m.hist);
    k_rs_scan<<<dim3(1), dim3(1024), 0, st>>>(m.count, m.hist);
    k_rs_scatter<<<dim3(tiles), dim3(kWave), 0, st>>>(kin, vin, m.count, shift, m.hist, kout, vout);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  // VALMOD_MSET_LDS_BUCKETS lowers the LDS bucket-map limit (0: always the global map; a test hook)
  const char* ev = getenv("VALMOD_MSET_LDS_BUCKETS");
  int64_t lds_max = ev && *ev ? atoll(ev) : kLdsBuckets;
  lds_max = lds_max < 0 ? 0 : (lds_max > kLdsBuckets ? kLdsBuckets : lds_max);
  k_set_greedy<<<dim3(1), dim3(kGreedyThreads), 0, st>>>(kin, vin, m.count, m.abl, m.excl_den, m.k, m.cap, m.n0,
                                                         lds_max, m.taken, m.bucket, m.out_count, m.out_off,
                                                         m.out_dist);
  return hipGetLastError();
}

}  // namespace valmod
