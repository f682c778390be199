/*
 * valmod.h - C ABI of the MI355X (gfx950) implementation of the hot path of
 * VALMOD, the variable-length motif and discord discovery method of
 * "Matrix Profile Goes MAD" (Linardi, Zhu, Palpanas, Keogh).
 *
 * What one run computes, for each series T of n points and every length L in
 * [l_min, l_max] (Problem "Variable-Length Motif Pair Discovery"; Problem
 * "Variable-Length Top-k m-th Discord Discovery" with m = 1):
 *   - the matrix profile MP_L and its index IP_L (Def. "Matrix profile"): for
 *     every window i, the z-normalised Euclidean distance (Eq. 6) to its nearest
 *     non-trivial neighbour and that neighbour's offset;
 *   - the variable-length matrix profile VALMP (Alg. updateVALMP): per offset, the
 *     smallest length-normalised distance d * sqrt(1/L) over all lengths, with
 *     its raw distance, length and neighbour;
 *   - per length, the top-k motif pairs and the top-k 1st discords, and across
 *     lengths the top-k motif pairs (from VALMP) and the discord ranking of
 *     Sec. "Comparing Discords of Different Lengths" (position-wise max of
 *     d / sqrt(L)).
 * Internally the profile at the smallest length is computed with the diagonal
 * dot-product recurrence (Alg. ComputeMatrixProfile) while keeping, per window,
 * the p candidates with the smallest lower bound (Eq. lowerBoundFinalFormula);
 * longer lengths reuse those partial profiles (Alg. ComputeSubMP) and recompute
 * only the windows whose bound test fails, so every MP_L is exact.
 *
 * Conventions (all offsets 0-based):
 *   N_L = n - L + 1 windows; trivial match iff |i - j| <= ceil(L / excl_den);
 *   population standard deviation (Eq. 6); a window is flat iff
 *   sigma <= flat_eps * max(1, |mu|), and flat windows are neither owners nor
 *   candidates (distance +inf, index -1); ties go to the smaller index.
 *
 * Memory ownership: the caller owns every device buffer (input series,
 * workspace, outputs); the plan owns host metadata and, from its first
 * valmod_run, per-lane HIP streams and events, a few bytes of pinned host
 * memory per lane and (graph mode) the instantiated graph, all released by
 * valmod_plan_free. No function of this library allocates device memory.
 * Return values are valmod_status codes; no exception crosses the ABI.
 * Argument errors are reported synchronously by valmod_plan / valmod_run;
 * errors found on the device (non-finite input) are written to a device status
 * word that valmod_run_status reads after the run has completed
 * (VALMOD_E_DEVICE).
 *
 * Threading: a plan may be used by one host thread and one stream at a time.
 */
#ifndef VALMOD_H
#define VALMOD_H

#include <stddef.h>
#include <stdint.h>

#ifndef VALMOD_API
#define VALMOD_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VALMOD_OK = 0,
  VALMOD_E_ARG = -1,       /* bad argument (null, out of range, inconsistent) */
  VALMOD_E_TOO_SHORT = -2, /* a series has no non-trivial pair at l_max */
  VALMOD_E_NOMEM = -3,     /* host allocation failed */
  VALMOD_E_HIP = -4,       /* a HIP runtime call failed */
  VALMOD_E_LAYOUT = -5,    /* sizes exceed the supported index range */
  VALMOD_E_DEVICE = -6,    /* error reported by a kernel (returned by valmod_run_status) */
  VALMOD_E_SCRATCH = -7    /* valmod_run_noalloc: the plan's workspace exceeds its static scratch */
} valmod_status;

typedef enum { VALMOD_F32 = 0, VALMOD_F64 = 1 } valmod_dtype;

/* Arithmetic of the diagonal recurrence. Statistics, lower bounds, the length
 * sweep and every reported distance are FP64 in both modes, and both modes
 * return the same exact results: the FP32 recurrence only selects candidates,
 * with a threshold widened by a rigorous bound of its rounding error per work
 * item; work items whose bound exceeds a limit run in FP64, and every selected
 * candidate is re-evaluated in FP64. The FP64 recurrence selects the same way,
 * with its own bound. The first length of each series starts with an FP64
 * matrix-profile pass whose neighbours seed its collecting pass. */
typedef enum {
  VALMOD_PREC_FP64 = 0,        /* recurrence in FP64 */
  VALMOD_PREC_FP32_REFRESH = 1 /* recurrence in FP32, restarted from FP64 dot products every R rows */
} valmod_precision;

/* Which of the two ways of getting MP_L for L > base is used. */
typedef enum {
  VALMOD_PATH_AUTO = 0,      /* cost model: row recompute of failing windows, or a full pass */
  VALMOD_PATH_FULL = 1,      /* a full diagonal pass at every length (test hook) */
  VALMOD_PATH_RECOMPUTE = 2  /* never a full pass after l_min (test hook) */
} valmod_path;

/* What the per-length update guarantees. */
typedef enum {
  VALMOD_MODE_EXACT = 0, /* every MP_L entry exact: every window whose bound test fails is recomputed */
  VALMOD_MODE_PAPER = 1  /* Alg. ComputeSubMP as published: only the failing windows whose bound is
                            below the best certified distance are recomputed (or a full pass when they
                            are many), so the motif of every length is exact while other MP_L entries
                            may be left uncomputed: index -2, distance = a lower bound of the entry */
} valmod_mode;

/* Maximum number of windows of one series (candidate indices are packed in 22 bits). */
#define VALMOD_MAX_WINDOWS ((int64_t)1 << 22)

typedef struct {
  int32_t num_series;       /* >= 1 */
  const int64_t* n;         /* host array [num_series]: points per series */
  const int32_t* l_min;     /* host array [num_series] */
  const int32_t* l_max;     /* host array [num_series], l_max >= l_min >= 4 */
  int32_t p;                /* partial-profile size (Alg. ComputeMatrixProfile); 0 = default 10 */
  int32_t k_motifs;         /* top-k motif pairs per length and across lengths, >= 1 */
  int32_t k_discords;       /* top-k discords per length and across lengths, >= 1 */
  int32_t excl_den;         /* exclusion zone ceil(L / excl_den); 0 = default 4 */
  double flat_eps;          /* flat-window threshold; 0 = default 2^-20 */
  int32_t dtype;            /* valmod_dtype of the input series */
  int32_t precision;        /* valmod_precision */
  int32_t refresh_R;        /* FP32 refresh interval R in rows: 0 = default (256, doubled up to 1024
                               while the anchor table exceeds its memory budget; valmod_autotune may
                               pick 256, 512 or 1024), else a multiple of 16 in [64, 8192]; the
                               rounding bound grows linearly with R */
  int32_t path;             /* valmod_path */
  int32_t device;           /* HIP device ordinal the plan runs on */
  int32_t lanes;            /* series processed concurrently (streams), 0 = default min(num_series, 16),
                               at most 64; each lane has its own workspace slice */
  int32_t graph;            /* 1: capture the whole run in a HIP graph on the first call and replay it on
                               later calls with the same buffers and stream; implies VALMOD_PATH_FULL
                               (VALMOD_PATH_RECOMPUTE is rejected); FP64 precision only */
  int32_t mode;             /* valmod_mode; VALMOD_MODE_PAPER needs VALMOD_PATH_AUTO and no graph */
  int32_t m_discords;       /* m of the Top-k m-th discords (0 or 1: only the 1st discords); m > 1 needs
                               m <= 16, m <= p, exact mode and no graph, and the mdiscord outputs.
                               With partial profiles the m-lists follow Alg. Topkm_nextLength: certified
                               from the profiles, pruned by the top-k cutoff, or recomputed */
  double mset_radius;       /* radius factor D of the motif sets (Sec. "Finding Motif Sets"): 0 = no
                               motif sets; else in (0, 1e6], and the mset outputs are required */
  int32_t mset_cap;         /* members stored per motif set, in [1, 2^20] when mset_radius > 0 (the
                               count of members is reported in full) */
} valmod_config;

typedef struct valmod_plan_s* valmod_plan_t;

/* Per-length diagnostic counters (stats[(L - l_min) * VALMOD_NSTATS + c]). */
enum {
  VALMOD_STAT_VALID = 0,      /* windows whose partial profile certified the minimum */
  VALMOD_STAT_FAILED = 1,     /* windows whose bound test failed */
  VALMOD_STAT_RECOMPUTED = 2, /* windows recomputed by a row scan */
  VALMOD_STAT_FULL_PASS = 3,  /* 1 if a full diagonal pass ran at this length */
  VALMOD_STAT_FLAT = 4,       /* flat windows at this length */
  VALMOD_STAT_APPENDS = 5,    /* candidates collected by the full pass (0 if none) */
  VALMOD_STAT_PASS_EVENTS = 6,/* wavefront steps of the diagonal pass that took its slow path */
  VALMOD_STAT_PASS_HITS = 7,  /* owner updates made by the diagonal pass */
  VALMOD_STAT_FP64_ITEMS = 8, /* FP32 path: work items whose rounding bound sent them to the FP64 kernel */
  VALMOD_STAT_PASSES = 9,     /* diagonal-pass launches at this length */
  VALMOD_STAT_PARTIAL = 10,   /* paper mode: profile entries left uncomputed (index -2) */
  /* m-th discords with partial profiles (Alg. Topkm_nextLength), 0 at lengths that build
     the m-lists with a full pass: */
  VALMOD_STAT_MTH_CERTIFIED = 11,  /* windows whose m best matches the partial profile certifies */
  VALMOD_STAT_MTH_RECOMPUTED = 12, /* windows whose m best matches a top-m row scan recomputes */
  VALMOD_STAT_MTH_PRUNED = 13,     /* uncertified windows the top-k cutoff leaves out of the
                                      m-th discord rankings (their best match stays exact) */
  VALMOD_STAT_OVERFLOWED = 14,     /* at a length that rebuilds the partial profiles: windows whose
                                      candidate list of the pass with p thresholds overflowed */
  VALMOD_NSTATS = 15
};

/*
 * Output buffers (device pointers, caller-allocated). A NULL pointer skips that
 * output (nothing is written there; what the run needs of it internally lives in
 * the workspace), except that the m-th discord outputs are required when
 * m_discords > 1 and the motif-set outputs when mset_radius > 0. Skipping
 * prof_dist / prof_idx saves n0 * nlen * 12 bytes per series.
 * For series s with N0 = n_s - l_min_s + 1 and nlen = l_max_s - l_min_s + 1,
 * element offsets come from valmod_series_layout; inside one series:
 *   prof_dist[t * N0 + i]  f64  MP_L[i] for L = l_min + t (+inf if none; +inf for i >= N_L)
 *   prof_idx [t * N0 + i]  i32  IP_L[i] (-1 if none; paper mode: -2 if not computed, and then
 *                               prof_dist holds a lower bound of MP_L[i])
 *   valmp_norm/valmp_dist[i] f64, valmp_len/valmp_idx[i] i32, i < N0 (len 0 / idx -1 if empty)
 *   motif_ab[(t * k_m + r) * 2 + {0,1}] i32 (a < b), motif_d[t * k_m + r] f64 (NaN / -1 unused)
 *   discord_on[(t * k_d + r) * 2 + {0,1}] i32 (offset, neighbour), discord_d[t * k_d + r] f64
 *   (paper mode: rankings use the computed entries only; the first motif of each length and the
 *   first global motif are exact, later ranks and the discords are over the computed entries)
 *   g_motif_abl[r * 3 + {0,1,2}] i32 (a, b, L), g_motif_d[r * 2 + {0,1}] f64 (d, d*sqrt(1/L))
 *   g_discord_onl[r * 3 + {0,1,2}] i32 (offset, neighbour, L), g_discord_d[r * 2 + {0,1}] f64 (d, d/sqrt(L))
 *   stats[t * VALMOD_NSTATS + c] i64
 *   with m = m_discords > 1 (Defs. m-th best match and Top-k m-th discord; j = 0..m-1 is the
 *   (j+1)-th best match, the neighbours may be trivial matches of each other):
 *   mdiscord_on[((t * m + j) * k_d + r) * 2 + {0,1}] i32 (offset, (j+1)-th neighbour),
 *   mdiscord_d[(t * m + j) * k_d + r] f64, g_mdiscord_onl[(j * k_d + r) * 3 + {0,1,2}] i32 (offset,
 *   neighbour, L), g_mdiscord_d[(j * k_d + r) * 2 + {0,1}] f64 (d, d/sqrt(L)); unused slots -1 / NaN
 *   with mset_radius = D > 0 (Def. data series motif set; Problem of variable-length motif sets
 *   discovery): one set per global motif pair r (a, b, L, d) of g_motif_*, taken in rank order, with
 *   radius D * d: the windows of length L whose z-normalised distance to a or to b is below the
 *   radius, in order of (distance to the nearer of a and b, offset), skipping a window that is a
 *   trivial match of a member already taken for this set or whose offset an earlier set of the
 *   series already holds (sets are disjoint by offset across lengths). Distances closer than
 *   D * d * 2^-36 count as equal. Flat windows are never members.
 *   mset_count[r] i32 (members, also beyond mset_cap), mset_off[r * mset_cap + i] i32 and
 *   mset_dist[r * mset_cap + i] f64 (raw distance to the nearer pair member) for i < min(count,
 *   mset_cap), -1 / NaN after; offsets: mset_count at the series' g_motif, the others at its mset
 */
typedef struct {
  double* prof_dist;
  int32_t* prof_idx;
  double* valmp_norm;
  double* valmp_dist;
  int32_t* valmp_len;
  int32_t* valmp_idx;
  int32_t* motif_ab;
  double* motif_d;
  int32_t* discord_on;
  double* discord_d;
  int32_t* g_motif_abl;
  double* g_motif_d;
  int32_t* g_discord_onl;
  double* g_discord_d;
  int64_t* stats;
  int32_t* mdiscord_on;    /* m_discords > 1 only (else ignored) */
  double* mdiscord_d;
  int32_t* g_mdiscord_onl;
  double* g_mdiscord_d;
  int32_t* mset_count;     /* mset_radius > 0 only (else ignored) */
  int32_t* mset_off;
  double* mset_dist;
} valmod_outputs;

/* Element counts of every output array over the whole batch. */
typedef struct {
  int64_t prof;       /* prof_dist, prof_idx */
  int64_t valmp;      /* valmp_* */
  int64_t motif;      /* motif_d (motif_ab holds 2x) */
  int64_t discord;    /* discord_d (discord_on holds 2x) */
  int64_t g_motif;    /* rows of g_motif_* (abl holds 3x, d 2x) */
  int64_t g_discord;  /* rows of g_discord_* */
  int64_t stats;      /* stats */
  int64_t series;     /* elements of the concatenated input series */
  int64_t mdiscord;   /* mdiscord_d (mdiscord_on holds 2x); 0 unless m_discords > 1 */
  int64_t g_mdiscord; /* rows of g_mdiscord_* */
  int64_t mset;       /* mset_off, mset_dist (g_motif * mset_cap); 0 unless mset_radius > 0 */
} valmod_sizes;

/* Element offsets of series s inside the concatenated input and each output. */
typedef struct {
  int64_t series;
  int64_t prof;
  int64_t valmp;
  int64_t motif;
  int64_t discord;
  int64_t g_motif;
  int64_t g_discord;
  int64_t stats;
  int64_t n, n0, nlen;
  int32_t l_min, l_max;
  int64_t mdiscord;
  int64_t g_mdiscord;
  int64_t mset;
} valmod_layout;

/* Validate a configuration and build a plan (host only; touches no GPU): the
 * inputs of Problem "Variable-Length Motif Pair Discovery" (series, l_min,
 * l_max, k) and of Problem "Variable-Length Top-k m-th Discord Discovery" (k, m),
 * plus the partial-profile size p of Alg. ComputeMatrixProfile. The
 * series are assigned to `lanes` by longest processing time first on the sum
 * over lengths of N_L^2; each lane runs its series one after another.
 * Errors: VALMOD_E_ARG (null pointers, num_series < 1, l_min < 4, l_max < l_min,
 * p < 0, k < 1, excl_den < 0, flat_eps < 0, unknown enum, lanes outside
 * [0, 64], graph not 0/1, graph with VALMOD_PATH_RECOMPUTE or with
 * VALMOD_PREC_FP32_REFRESH, unknown mode, paper mode with another path than
 * VALMOD_PATH_AUTO or with graph, m_discords or motif-set fields out of
 * range), VALMOD_E_TOO_SHORT
 * (n - l_max + 1 <= ceil(l_max / excl_den) + 1: no non-trivial pair),
 * VALMOD_E_LAYOUT (more than VALMOD_MAX_WINDOWS windows), VALMOD_E_NOMEM. */
VALMOD_API valmod_status valmod_plan(const valmod_config* cfg, valmod_plan_t* out);

/* Device workspace the caller must pass to valmod_run (bytes, 256-aligned base):
 * statistics, recurrence inputs, anchor table, partial profiles (Alg.
 * ComputeMatrixProfile, Alg. ComputeSubMP) and the last profile rows of each
 * lane. 0 for a NULL plan. */
VALMOD_API size_t valmod_workspace_bytes(valmod_plan_t plan);

/* Output element counts of the whole batch (the outputs of Problems "Variable-Length
 * Motif Pair Discovery" and "Variable-Length Top-k m-th Discord Discovery");
 * VALMOD_E_ARG if plan or out is NULL. */
VALMOD_API valmod_status valmod_output_sizes(valmod_plan_t plan, valmod_sizes* out);

/* Element offsets of series s (0 <= s < num_series) inside the concatenated input
 * and every output; VALMOD_E_ARG otherwise. */
VALMOD_API valmod_status valmod_series_layout(valmod_plan_t plan, int32_t s, valmod_layout* out);

/*
 * Run the plan (Alg. VALMOD over every series: the matrix profile at l_min by
 * Alg. ComputeMatrixProfile, the longer lengths by Alg. ComputeSubMP, VALMP by
 * Alg. updateVALMP, the rankings of Sec. "Comparing Motifs of Different Lengths"
 * and Alg. UpdateVariableLengthDiscords). d_series: device array of the
 * concatenated series in the configured dtype (series s starts at element
 * valmod_layout.series). d_workspace: device buffer of valmod_workspace_bytes(plan)
 * bytes, 256-byte aligned, contents irrelevant on entry. d_out: struct (host
 * memory) of device pointers; NULL members skip their output. stream: a
 * hipStream_t (passed as void*; NULL = default stream).
 * The call enqueues the run on `stream` and returns without waiting for it to
 * finish: the lanes' streams start after the work already on `stream`, and
 * `stream` waits for all of them. Plans with partial profiles (path AUTO or
 * RECOMPUTE, or paper mode) wait inside the call at lengths whose next step
 * depends on device counters (the number of windows whose bound test failed);
 * full-path and graph plans never wait. The outputs are complete, and the run's
 * device status is known, once valmod_run_status has returned. In graph mode the
 * first call captures the run (lanes included) into a HIP graph and launches it;
 * later calls with the same d_series, d_workspace, output pointers and stream
 * replay it. One plan must not be used by two calls at the same time, and a
 * second run of a plan may be enqueued before the first one's status is read
 * (valmod_run_status then reports the last one). Errors (synchronous):
 * VALMOD_E_ARG (null plan/series/workspace/out, unaligned workspace, missing
 * m-th discord or motif-set outputs), VALMOD_E_HIP (a launch or runtime call
 * failed).
 */
VALMOD_API valmod_status valmod_run(valmod_plan_t plan, const void* d_series, void* d_workspace,
                         const valmod_outputs* d_out, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): valmod_run with the
 * workspace in a static device array of VALMOD_NOALLOC_SCRATCH_BYTES (64 MiB)
 * that the library holds on every GPU it runs on until the process ends. The
 * caller still passes the input series and the outputs (NULL members skip their
 * output, as for valmod_run). The call allocates nothing: no device or pinned
 * memory, no streams or events; every lane's series run in turn on `stream`,
 * with a full diagonal pass at every length (partial profiles take host
 * decisions, so they are off; in exact mode the outputs are the same) and no
 * pass timing. The call enqueues and returns; valmod_run_status waits and reads
 * the device status word. All calls on one GPU share its array and it keeps the
 * last call's contents (each run clears what it reads first), so calls that
 * overlap on one GPU race: serialise them. Errors: VALMOD_E_SCRATCH when
 * valmod_workspace_bytes(plan) exceeds the array, VALMOD_E_ARG (null arguments,
 * paper mode, missing m-th discord or motif-set outputs), VALMOD_E_HIP.
 */
#define VALMOD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
VALMOD_API valmod_status valmod_run_noalloc(valmod_plan_t plan, const void* d_series, const valmod_outputs* d_out,
                                            void* stream);

/*
 * Wait for the last run enqueued by valmod_run or valmod_run_noalloc on this plan (synchronising
 * `stream` first when it is not NULL) and return its status: VALMOD_OK,
 * VALMOD_E_DEVICE (the input held non-finite values; the device status word of a
 * lane was set) or VALMOD_E_HIP. Also makes valmod_last_pass_timing reflect that
 * run. Without a pending run it returns the status of the last one read
 * (VALMOD_OK before any). VALMOD_E_ARG for a NULL plan.
 */
VALMOD_API valmod_status valmod_run_status(valmod_plan_t plan, void* stream);

/*
 * Autotuner: choose the diagonal-pass geometry and the partial-profile size p
 * empirically, on the series with the most work (the pass geometry of Alg.
 * ComputeMatrixProfile's recurrence; p of Alg. ComputeMatrixProfile and Alg.
 * ComputeSubMP). Stage 1: FP64 plans try segment heights of 1x, 2x and 4x the
 * default; FP32 plans without a fixed refresh_R try R = 256, 512 and 1024 with 8
 * and 4 diagonals per lane (4 only unless VALMOD_PASS_K32 fixes it); each
 * candidate is timed on three lengths at the start and three at the end of the
 * range on the full path. Stage 2 (exact mode with partial profiles): p, p/2 and
 * p/4 are timed on the first four lengths with the plan's own path, and against
 * them a run without partial profiles (a full pass at every length; the outputs
 * depend on neither choice in exact mode). Every measurement is the second of two runs,
 * and the fastest candidate whose workspace fits in valmod_workspace_bytes (as it
 * was before the call) is kept: the plan's workspace requirement can only shrink.
 * Arguments are those of valmod_run (same buffers; d_out may be NULL: the tuning
 * runs write no output). The call waits for its runs. chosen (optional, host
 * int32[3]): segment height, diagonals per lane and p of the tuned series (p = 0:
 * partial profiles off; the current ones when nothing was tuned). Errors: those
 * of valmod_run.
 */
VALMOD_API valmod_status valmod_autotune(valmod_plan_t plan, const void* d_series, void* d_workspace,
                                         const valmod_outputs* d_out, void* stream, int32_t* chosen);

/* Release a plan and the streams, events, pinned words and graph it holds
 * (NULL is ignored). The plan's last run must have completed. */
VALMOD_API void valmod_plan_free(valmod_plan_t plan);

/* Human-readable name of a status code (static string; "unknown status" for
 * codes outside valmod_status). */
VALMOD_API const char* valmod_status_str(int status);

/* Milliseconds spent in the diagonal-pass kernel of the plan's precision during
 * the last valmod_run (full-grid launches only: FP64 mode, every pass; FP32
 * mode, the FP32 collecting passes, not the FP64 pass of the first length nor
 * the FP64 re-runs of listed work items), measured with HIP events that each
 * launch records itself at kernel start and end on its lane's stream, and the
 * number of those launches and of the cells they covered, as of the last
 * valmod_run_status. In graph mode: the time of the whole replay, as one launch.
 * Measurement hook of the diagonal pass of Alg. ComputeMatrixProfile. */
VALMOD_API valmod_status valmod_last_pass_timing(valmod_plan_t plan, double* ms, int64_t* launches,
                                      int64_t* cells);

/*
 * Rounding bound used by the diagonal pass for one work item, in correlation
 * units: the largest |rho computed - rho| of the recurrence (the dot-product
 * update of Alg. ComputeMatrixProfile in co-moment form) over an item of H rows
 * at length L, in FP32 (precision VALMOD_PREC_FP32_REFRESH; includes the
 * rounding of the FP32 filter's own difference) or FP64 (VALMOD_PREC_FP64),
 * with phi = (max sw / min sw)_rows (max sw / min sw)_cols and psi =
 * (max|df|_rows max|dg|_cols + max|dg|_rows max|df|_cols) / (min sw_rows min sw_cols)
 * and xi = (max|df|_rows + max|df|_cols) max|mu| / (min sw_rows min sw_cols)
 * over the item's windows (sw = sigma sqrt(L); df, dg the recurrence inputs
 * df_i = (x_{i+L} - x_i) / 2, dg_i = (x_{i+L} - mu_{i+1}) + (x_i - mu_i)).
 * Host function (no device work); NaN for H < 1, L < 1, negative phi, psi or
 * xi, or an unknown precision.
 */
VALMOD_API double valmod_rounding_bound(int32_t precision, int64_t H, int32_t L, double phi, double psi,
                                        double xi);

#ifdef __cplusplus
}
#endif

#endif /* VALMOD_H */
