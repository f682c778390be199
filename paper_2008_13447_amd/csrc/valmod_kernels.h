// Launch wrappers of the VALMOD kernels (host side, no allocation, asynchronous).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace valmod {

constexpr int kPassKMax = 8;  // largest supported diagonals-per-lane of the pass (4 or 8)

// Slots of the device counter block of a run (64-bit each). The per-length ones
// are recorded and cleared by launch_record_stats at the end of every length.
enum CounterSlot {
  CNT_ERR = 0,       // error flag (non-finite input)
  CNT_NFLAT = 1,     // flat windows at this length
  CNT_EV_STEPS = 2,  // pass wavefront steps that took the slow path
  CNT_EV_HITS = 3,   // pass queue entries
  CNT_APPENDS = 4,   // candidates collected by the collecting pass
  CNT_NFAIL = 5,     // owners in the recompute list
  CNT_VALID = 6,     // owners certified by the sweep
  CNT_HARD = 7,      // FP32 work items listed for the FP64 kernel
  CNT_BIG = 8,       // owners listed for the wavefront-per-owner merge
  CNT_MINDIST = 9,   // paper mode: minimum certified distance (bits of a double)
  CNT_MINLB = 10,    // paper mode: minimum bound of the failing owners (bits of a double)
  CNT_NREC = 11,     // paper mode: owners listed for the row recompute
  CNT_NPART = 12,    // paper mode: owners left partial
  CNT_RFLAT = 13,    // largest sigma_b / sigma_L of the windows flat at the base length but not at L (bits of a double)
  CNT_MOPEN = 14,    // m-th discords: owners whose m-list the partial profiles do not certify
  CNT_OVER = 15,     // owners whose list overflowed in the last rebuild's collecting pass with p thresholds
  CNT_MREC = 16,     // m-th discords: owners listed for the top-m row recompute
  CNT_MCERT = 17,    // m-th discords: owners whose m-list the partial profiles certify
  CNT_MPRUNED = 18,  // m-th discords: uncertified owners left out by the top-k cutoff
  CNT_WORDS = 32
};

struct PassLaunch {
  const double *xs, *mu, *df, *dg, *invn;
  const float* sw32;
  const float *df32, *dg32, *inv32;  // FP32 recurrence inputs
  double* thr;
  float* thr32;
  const int32_t* items;  // optional work-item list (FP64 re-run of items the FP32 bound rejects)
  int64_t nitems;        // grid size for the list (upper bound of the count)
  const unsigned long long* nitems_dev;  // device count of listed items
  const float* delta;    // rounding bound per work item of the pass's precision (null: none)
  float delta_max;       // items with a larger bound are skipped (left to the FP64 kernel)
  bool fp32;
  uint64_t* best;
  uint32_t* cnt;
  int32_t* buf;
  int64_t cap;
  const double* anc;
  const double* A;
  int64_t anc_stride;
  unsigned long long* events;
  int64_t N, e, H, dstart;
  int L;
  int K;  // diagonals per lane: 8 (FP64 also 4)
  bool append;
  bool grow;  // the pass also moves the anchor table on to length L + 1 (its last read at L)
  // optional: events recorded by the full-grid launch itself (start and end of
  // the kernel), so timing it adds no marker between it and its neighbours
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

struct PassGrid {
  int64_t bands = 0, segs = 0, cells = 0;
};

// Work decomposition of the diagonal pass over the upper triangle j - i > e.
PassGrid pass_grid(int64_t N, int64_t e, int64_t dstart, int K, int64_t H);

hipError_t launch_anchor(const double* xs, int64_t n, int L, bool init, int64_t H, int64_t dstart, int64_t segs,
                         int64_t stride, int64_t ncols, double* anc, hipStream_t st);

hipError_t launch_convert(const void* in, int dtype, int64_t n, int64_t npad, double* xs, int* err,
                          hipStream_t st);
// per-window inputs of one length: statistics, recurrence inputs and (df32 != null)
// the FP32 copies and the per-64-window extrema of the FP32 rounding bound
struct WindowPrep {
  const double* xs;
  int64_t N;
  int L;
  int first;  // 1: sums formed directly (first length of a series)
  double flat_eps;
  const double *A_in, *B_in;  // sums of the previous length (unused when first)
  double *A_out, *B_out;      // sums of this length
  double *mu, *sig, *invn;
  uint8_t* flat;
  unsigned long long* nflat;
  double *df, *dg;
  float* sw32;
  float *df32, *dg32, *inv32;                    // FP32 path (null: none)
  float *bsw_max, *bsw_min, *bdf_max, *bdg_max, *bmu_max;  // per-64-window extrema of the rounding bounds
  // partial profiles at base b (null: none): windows flat at b (hflat) but not at L
  // raise *rflat to their sigma_b / sigma_L (hsig: sigma at b)
  const uint8_t* hflat;
  const double* hsig;
  unsigned long long* rflat;
};
hipError_t launch_window_prep(const WindowPrep& w, hipStream_t st);
hipError_t launch_seed_mp(const double* xs, const double* mu, const double* invn, const uint8_t* flat,
                          const int32_t* prev_idx, int64_t N, int L, int64_t e, uint64_t* best,
                          double* thr, float* thr32, hipStream_t st);
hipError_t launch_pass(const PassLaunch& p, hipStream_t st);
// Rounding bounds of the diagonal pass per work item: delta64 (FP64 recurrence)
// always; with delta32 non-null also the FP32 bound, and the items whose FP32
// bound exceeds delta_max are listed in `hard` for the FP64 kernel.
hipError_t launch_item_bounds(const float* bsw_max, const float* bsw_min, const float* bdf_max, const float* bdg_max,
                              const float* bmu_max, int64_t N, int64_t e, int64_t dstart, int K, int64_t H, int L,
                              float delta_max,
                              float* delta64, float* delta32, int32_t* hard, unsigned long long* nhard,
                              hipStream_t st);
// Profile row of one length from the best keys into ring_dist / ring_idx and,
// when non-null, prof_dist / prof_idx (also +inf / -1 for the entries
// N .. N0 - 1); the VALMP update.
hipError_t launch_finalize(const double* xs, const double* mu, const double* sig, const uint64_t* best,
                           int64_t N, int64_t N0, int L, double* ring_dist, int32_t* ring_idx, double* prof_dist,
                           int32_t* prof_idx, double* valmp_norm, double* valmp_dist, int32_t* valmp_len,
                           int32_t* valmp_idx, hipStream_t st);
// Writes one stats row (host-known values and the per-length device counters;
// `recomputed`: 0 none, 1 the recompute list (CNT_NFAIL), 2 the paper-mode list
// (CNT_NREC)) and clears the per-length counters.
hipError_t launch_record_stats(unsigned long long* cnt, int64_t* row, int full_pass, int64_t valid,
                               int64_t failed, int recomputed, int64_t passes, int rebuilt, hipStream_t st);
// sets n consecutive counters to v (a kernel, so that the sequence stays capturable)
hipError_t launch_fill_counters(unsigned long long* p, int n, unsigned long long v, hipStream_t st);
inline hipError_t launch_zero_counters(unsigned long long* p, int n, hipStream_t st) {
  return launch_fill_counters(p, n, 0ull, st);
}
hipError_t launch_valmp_init(int64_t N0, double* norm, double* dist, int32_t* len, int32_t* idx,
                             hipStream_t st);
hipError_t launch_rankings(const double* prof_dist, const int32_t* prof_idx, int64_t N0, int64_t n, int l_min,
                           int nlen, int excl_den, int km, int kd, int32_t* motif_ab, double* motif_d,
                           int32_t* discord_on, double* discord_d, hipStream_t st);
hipError_t launch_global_rank(const double* valmp_norm, const double* valmp_dist, const int32_t* valmp_len,
                              const int32_t* valmp_idx, int64_t N0, const int32_t* discord_on,
                              const double* discord_d, int nlen, int l_min, int excl_den, int km, int kd,
                              int32_t* g_motif_abl, double* g_motif_d, int32_t* g_discord_onl,
                              double* g_discord_d, hipStream_t st);

// partial distance profiles (valmod_heap.hip)
// thr32 (optional): FP32 copy of each written threshold, rounded down
// thresholds of a rebuild from the partial profiles it replaces (after the sweep):
// thrp per owner, then the collecting thresholds raised to them
hipError_t launch_profile_threshold(const double* A, const double* invn, const uint8_t* flat, const int32_t* hc,
                                    const double* hS, const int32_t* hn, int p, int64_t N, int L, int64_t e,
                                    double margin, double* thrp, hipStream_t st);
hipError_t launch_tighten_threshold(const double* thrp, int64_t N, double* thr, float* thr32, hipStream_t st);
hipError_t launch_seed_append(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                              const int32_t* src, int64_t N, int L, int64_t e, int p, int D, double margin,
                              int best_exact, double* thr, float* thr32, uint32_t* cnt, int32_t* fail,
                              unsigned long long* nfail, hipStream_t st);
hipError_t launch_merge(const double* xs, const double* A, const double* invn, const double* sig, const uint8_t* flat,
                        const double* thr, const uint32_t* cnt, const int32_t* buf, int64_t cap, int64_t N, int L,
                        int p, int keep, double margin, int best_exact, int32_t* hc, double* hS, int32_t* hn,
                        double* hbound, double* hsig, uint8_t* hflat, uint64_t* best, int32_t* fail,
                        unsigned long long* nfail, int32_t* big, unsigned long long* nbig, unsigned long long* nappend,
                        unsigned long long* nover, hipStream_t st);
// lbm, min_dist, min_lb: optional (paper mode)
hipError_t launch_sweep(const double* xs, const double* A, const double* invn, const double* sig, const uint8_t* flat,
                        int64_t N, int L, int64_t e, int p, int base, const int32_t* hc, double* hS, const int32_t* hn,
                        const double* hbound, const double* hsig, const unsigned long long* rflat, double margin,
                        uint64_t* best, int32_t* fail, unsigned long long* nfail, unsigned long long* nvalid,
                        double* lbm, unsigned long long* min_dist, unsigned long long* min_lb, hipStream_t st);
hipError_t launch_split_fail(const int32_t* fail, const unsigned long long* nfail, int64_t max_listed,
                             const double* lbm, const unsigned long long* limit, int all_partial, int32_t* rec,
                             unsigned long long* nrec, int32_t* part, unsigned long long* npart, hipStream_t st);
hipError_t launch_mark_partial(const int32_t* part, const unsigned long long* npart, int64_t max_listed,
                               const double* lbm, double* prof_dist, int32_t* prof_idx, hipStream_t st);
// the list length is read on the device (nfail); max_listed bounds it
hipError_t launch_recompute(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                            const int32_t* fail, const unsigned long long* nfail, int64_t max_listed, int64_t N,
                            int L, int64_t e, uint64_t* best, hipStream_t st);
// m-th best matches: top-m row recompute of the listed owners (keys: scratch of
// m keys per window), the j-th best-match distances of every owner, their
// rankings per length and across lengths
hipError_t launch_recompute_topm(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                 const int32_t* fail, const unsigned long long* nfail, int64_t max_listed, int64_t N,
                                 int L, int64_t e, int m, int p, uint64_t* keys, int32_t* hc, double* hS, int32_t* hn,
                                 uint64_t* best, bool mfma, hipStream_t st);
hipError_t launch_mth_values(const double* A, const double* invn, const uint8_t* flat, const int32_t* hc,
                             const double* hS, const int32_t* hn, int p, int m, int64_t N, int64_t N0, int L,
                             double* vals, int32_t* nn, hipStream_t st);
// emul: the exclusion zone is emul times the zone of length L (2 gives the
// pruning cutoff of the m-th discords)
hipError_t launch_mth_rankings(const double* vals, const int32_t* nn, int64_t N0, int64_t n, int L, int m,
                               int excl_den, int kd, int32_t* on, double* d, hipStream_t st, int emul = 1);
// m-th discords from the partial profiles (Alg. Topkm_nextLength): selection and
// certification of every owner's m best stored candidates, the pruning cutoff,
// and the top-m row recompute of the owners it cannot exclude
struct MthSelect {
  const double *A, *invn, *sig;
  const uint8_t* flat;
  const int32_t *hc, *hn;
  const double *hS, *hbound, *hsig;
  const unsigned long long* rflat;  // CNT_RFLAT (read unless fresh)
  int fresh;                        // the partial profiles were rebuilt at this length
  int p, m;
  int64_t N, N0;
  int L;
  int64_t e;
  int base;
  double margin;
  double* vals;  // j-th best-match distances, column j at j * N0
  int32_t* nn;
  double* ub;    // upper bounds of the uncertified owners' distances (same layout)
  uint8_t* mstate;
  unsigned long long* n_open;
};
hipError_t launch_mth_select(const MthSelect& a, hipStream_t st);
hipError_t launch_mth_prune(const uint8_t* mstate, const double* ub, const double* tau_d, int64_t N, int64_t N0,
                            int m, int kd, int best_exact, int32_t* mlist, unsigned long long* nmlist, int32_t* fail,
                            unsigned long long* nfail, unsigned long long* ncert, unsigned long long* npruned,
                            hipStream_t st);
hipError_t launch_recompute_topm_keys(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                      const int32_t* list, const unsigned long long* nlist, int64_t max_listed,
                                      int64_t N, int64_t N0, int L, int64_t e, int m, uint64_t* keys, uint64_t* best,
                                      double* vals, int32_t* nn, bool mfma, hipStream_t st);
hipError_t launch_mth_global(const int32_t* on, const double* d, int nlen, int l_min, int m, int kd,
                             int32_t* g_onl, double* g_d, hipStream_t st);
// motif sets grown from the global top-k motif pairs of one series (valmod_sets.hip)
struct MotifSetLaunch {
  const double* xs;       // padded FP64 series
  int64_t n, n0;          // points, windows at the smallest length
  const int32_t* abl;     // k rows (a, b, L), a < 0 for an unused rank
  const double* gd;       // k rows (d, d / sqrt(L))
  int k;                  // pairs (<= 64)
  double D;               // radius factor
  int excl_den;
  double flat_eps;
  int64_t cap;            // members stored per set
  int64_t cand_cap;       // candidate capacity: k * n0
  double* meta;           // 5 * 64 doubles
  uint32_t* count;        // 1 + k words: candidate count, then candidates per set
  uint64_t *keys0, *keys1;
  double *vals0, *vals1;  // cand_cap each
  uint32_t* hist;         // motif_sets_hist_words(cand_cap)
  uint64_t* taken;        // (n0 + 63) / 64 words
  uint32_t* bucket;       // n0 / 2 + 2 entries
  int32_t* out_count;     // k
  int32_t* out_off;       // k * cap
  double* out_dist;       // k * cap
};
size_t motif_sets_hist_words(int64_t cand_cap);
hipError_t launch_motif_sets(const MotifSetLaunch& m, hipStream_t st);
// Hankel-block contractions on FP64 MFMA (valmod_mfma.hip): the anchor table of
// the first length, and the exact row recompute of the listed owners
hipError_t launch_anchor_mfma(const double* xs, int64_t n, int L, int64_t H, int64_t dstart, int64_t segs,
                              int64_t stride, int64_t ncols, double* anc, hipStream_t st);
hipError_t launch_recompute_mfma(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                 const int32_t* list, const unsigned long long* nlist, int64_t max_listed, int64_t N,
                                 int L, int64_t e, uint64_t* best, hipStream_t st);
// round jr of the top-m recompute on matrix cores: out[o * m + jr] = the smallest
// key above out[o * m + jr - 1] (must be empty before the round)
hipError_t launch_recompute_round_mfma(const double* xs, const double* A, const double* invn, const uint8_t* flat,
                                       const int32_t* list, const unsigned long long* nlist, int64_t max_listed,
                                       int64_t N, int L, int64_t e, int m, int jr, uint64_t* out, hipStream_t st);
// copies best keys into an int32 index array (-1 for empty keys)
hipError_t launch_keys_to_idx(const uint64_t* best, int64_t N, int32_t* idx, hipStream_t st);

}  // namespace valmod
