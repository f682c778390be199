/*
 * CPU FP64 brute-force oracle for variable-length motif and discord discovery
 * (VALMOD, "Matrix Profile Goes MAD").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link or call this
 * file; only the test-suite, the smoke check and the CPU baseline of the bench
 * use it. It shares no code with the HIP implementation.
 *
 * Everything is computed from the definitions, slowly and in double precision:
 *   - window mean / population standard deviation by two passes (the sigma of
 *     Eq. (6) is sqrt(ss/l - mu^2), i.e. the population deviation);
 *   - z-normalised Euclidean distance (Def. "Data series motif pair") by direct
 *     differences of the z-normalised windows, never by the closed form;
 *   - distance profile / matrix profile / matrix-profile index (Defs. "Distance
 *     profile", "Matrix profile") by a full scan of every non-trivial candidate;
 *   - the variable-length matrix profile update of Alg. updateVALMP;
 *   - length-normalised rankings (Sec. "Comparing Motifs of Different Lengths",
 *     Sec. "Comparing Discords of Different Lengths").
 *
 * Readings taken where the paper is silent or ambiguous (listed in full in the
 * design notes of the repository):
 *   - trivial match iff |i - j| <= ceil(L / excl_den) (exclusion zone; the text
 *     says l/2, the workloads use l/4);
 *   - a window is flat iff sigma <= flat_eps * max(1, |mu|); flat windows are
 *     neither owners nor candidates (distance +inf, index -1); the flat rule is
 *     a reporting convention, so the lower bound of a window that is flat at the
 *     base length still uses its real correlation there (0 only when it is
 *     exactly constant);
 *   - ties in a distance profile go to the smallest candidate index;
 *   - the VALMP update compares length-normalised distances, strictly;
 *   - top-k motifs per length: pairs (i, IP[i]) sorted by (d, min, max), accepted
 *     greedily unless an endpoint is within the exclusion zone of an accepted
 *     endpoint;
 *   - top-k discords per length: offsets sorted by (MP descending, index
 *     ascending), accepted greedily with the same exclusion rule;
 *   - cross-length discords: position-wise max of d / sqrt(L), strict, so the
 *     shorter length wins ties;
 *   - cross-length motifs: VALMP entries sorted by (normalised d, length, i),
 *     endpoints trivial iff within ceil(max(La, Lb) / excl_den).
 *
 * Parity pins: every function here is checked by the CPU tests against values
 * fixed by the paper or by mathematics (closed form of Eq. (6), symmetry, the
 * lower bound of Eq. (lowerBoundFinalFormula) never exceeding the true
 * distance, rank preservation, affine invariance, brute force with another
 * library on tiny inputs, planted motif / discord recovery, Example 2). The
 * flat rule and the greedy top-k rules are definitions of this build: parity
 * unpinned beyond their special cases (top-1 motif = the motif pair, top-1
 * discord = the 1st discord). oracle_mth_rows / oracle_mth_discords follow the
 * definitions of the m-th best match and of the Top-k m-th discord, and
 * oracle_motif_sets the definition of the data series motif set (both pinned
 * against an independent brute force).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_EXPORT __attribute__((visibility("default")))

static int64_t excl_zone(int64_t L, int64_t den) { return (L + den - 1) / den; }

static int resolve_threads(int nthreads) {
  if (nthreads > 0) return nthreads;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  return c > 0 ? (int)c : 1;
}

/* Mean and population standard deviation of every window of length L, by two
 * passes; flat rule as documented above. */
ORACLE_EXPORT void oracle_stats(const double* x, int64_t n, int64_t L, double flat_eps,
                                double* mu, double* sigma, uint8_t* flat) {
  int64_t N = n - L + 1;
  for (int64_t i = 0; i < N; i++) {
    double s = 0.0;
    for (int64_t k = 0; k < L; k++) s += x[i + k];
    double m = s / (double)L;
    double v = 0.0;
    for (int64_t k = 0; k < L; k++) {
      double t = x[i + k] - m;
      v += t * t;
    }
    double sd = sqrt(v / (double)L);
    mu[i] = m;
    sigma[i] = sd;
    flat[i] = sd <= flat_eps * fmax(1.0, fabs(m)) ? 1 : 0;
  }
}

/* Squared z-normalised Euclidean distance of windows i and j (both non-flat),
 * by direct differences of the z-normalised values. */
static double sqdist(const double* x, int64_t L, int64_t i, int64_t j, const double* mu,
                     const double* sigma) {
  double acc = 0.0;
  for (int64_t k = 0; k < L; k++) {
    double zi = (x[i + k] - mu[i]) / sigma[i];
    double zj = (x[j + k] - mu[j]) / sigma[j];
    double t = zi - zj;
    acc += t * t;
  }
  return acc;
}

ORACLE_EXPORT double oracle_pair_dist(const double* x, int64_t n, int64_t L, int64_t i, int64_t j,
                                      double flat_eps) {
  int64_t N = n - L + 1;
  if (i < 0 || j < 0 || i >= N || j >= N) return NAN;
  double* mu = (double*)malloc(sizeof(double) * N);
  double* sg = (double*)malloc(sizeof(double) * N);
  uint8_t* fl = (uint8_t*)malloc(N);
  oracle_stats(x, n, L, flat_eps, mu, sg, fl);
  double d = (fl[i] || fl[j]) ? INFINITY : sqrt(sqdist(x, L, i, j, mu, sg));
  free(mu);
  free(sg);
  free(fl);
  return d;
}

/* Pearson correlation of two non-flat windows, directly from z-normalised values. */
static double pearson(const double* x, int64_t L, int64_t i, int64_t j, const double* mu,
                      const double* sigma) {
  double acc = 0.0;
  for (int64_t k = 0; k < L; k++)
    acc += ((x[i + k] - mu[i]) / sigma[i]) * ((x[j + k] - mu[j]) / sigma[j]);
  return acc / (double)L;
}

typedef struct {
  const double* x;
  int64_t L, N, e;
  const double *mu, *sigma;
  const uint8_t* flat;
  const int64_t* rows;
  int64_t nrows;
  double* dist;
  int64_t* idx;
  int64_t next; /* shared work counter */
  pthread_mutex_t lock;
} profile_job;

static void profile_one(profile_job* J, int64_t r) {
  int64_t i = J->rows ? J->rows[r] : r;
  double best = INFINITY;
  int64_t bi = -1;
  if (i >= 0 && i < J->N && !J->flat[i]) {
    for (int64_t j = 0; j < J->N; j++) {
      if (J->flat[j]) continue;
      int64_t dd = i > j ? i - j : j - i;
      if (dd <= J->e) continue; /* trivial match */
      double s = sqdist(J->x, J->L, i, j, J->mu, J->sigma);
      if (s < best) { /* strict: ties keep the smallest j */
        best = s;
        bi = j;
      }
    }
  }
  J->dist[r] = bi >= 0 ? sqrt(best) : INFINITY;
  J->idx[r] = bi;
}

static void* profile_worker(void* arg) {
  profile_job* J = (profile_job*)arg;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    int64_t r0 = J->next;
    J->next += 1;
    pthread_mutex_unlock(&J->lock);
    if (r0 >= J->nrows) break;
    int64_t r1 = r0 + 1 < J->nrows ? r0 + 1 : J->nrows;
    for (int64_t r = r0; r < r1; r++) profile_one(J, r);
  }
  return NULL;
}

static void run_profile(profile_job* J, int nthreads) {
  nthreads = resolve_threads(nthreads);
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  J->next = 0;
  pthread_mutex_init(&J->lock, NULL);
  for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, profile_worker, J);
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J->lock);
}

/* Matrix-profile entries (distance and index of the nearest non-trivial
 * neighbour) of the owners listed in rows[0..nrows) at length L. rows == NULL
 * means every owner 0..N-1 (then nrows must be N). */
ORACLE_EXPORT int oracle_profile_rows(const double* x, int64_t n, int64_t L, int64_t excl_den,
                                      double flat_eps, const int64_t* rows, int64_t nrows,
                                      double* dist, int64_t* idx, int nthreads) {
  int64_t N = n - L + 1;
  if (L < 2 || N < 1 || excl_den < 1) return -1;
  double* mu = (double*)malloc(sizeof(double) * N);
  double* sg = (double*)malloc(sizeof(double) * N);
  uint8_t* fl = (uint8_t*)malloc(N);
  oracle_stats(x, n, L, flat_eps, mu, sg, fl);
  profile_job J;
  J.x = x;
  J.L = L;
  J.N = N;
  J.e = excl_zone(L, excl_den);
  J.mu = mu;
  J.sigma = sg;
  J.flat = fl;
  J.rows = rows;
  J.nrows = rows ? nrows : N;
  J.dist = dist;
  J.idx = idx;
  run_profile(&J, nthreads);
  free(mu);
  free(sg);
  free(fl);
  return 0;
}

/* Lower bound of the distance of owner o and candidate c at length L, from
 * their base-length-b correlation (Eq. lowerBoundFinalFormula) and the owner's
 * sigma ratio (rank-preservation remark). Flat candidate at b: correlation
 * taken as 0; flat owner at b: 0; flat owner at L: +inf. */
ORACLE_EXPORT double oracle_lb(const double* x, int64_t n, int64_t o, int64_t c, int64_t b,
                               int64_t L, double flat_eps) {
  int64_t Nb = n - b + 1, NL = n - L + 1;
  if (o < 0 || c < 0 || o >= NL || c >= NL || L < b) return NAN;
  double* mu = (double*)malloc(sizeof(double) * Nb);
  double* sg = (double*)malloc(sizeof(double) * Nb);
  uint8_t* fl = (uint8_t*)malloc(Nb);
  double* muL = (double*)malloc(sizeof(double) * NL);
  double* sgL = (double*)malloc(sizeof(double) * NL);
  uint8_t* flL = (uint8_t*)malloc(NL);
  oracle_stats(x, n, b, flat_eps, mu, sg, fl);
  oracle_stats(x, n, L, flat_eps, muL, sgL, flL);
  double out;
  if (flL[o]) {
    out = INFINITY;
  } else if (fl[o]) {
    out = 0.0;
  } else {
    /* Eq. lowerBoundFinalFormula holds for any candidate shape: a window that
     * the flat rule excludes still has a correlation unless it is exactly
     * constant (then the minimising constant vector gives rho+ = 0) */
    double q = sg[c] > 0.0 ? pearson(x, b, o, c, mu, sg) : 0.0;
    double qp = q > 0.0 ? q : 0.0;
    double base = 1.0 - qp * qp;
    if (base < 0.0) base = 0.0;
    out = sqrt((double)b * base) * sg[o] / sgL[o];
  }
  free(mu);
  free(sg);
  free(fl);
  free(muL);
  free(sgL);
  free(flL);
  return out;
}

/* Direct distances of listed (i, j) pairs at length L (NaN for out-of-range,
 * +inf if either window is flat), with the statistics formed once. */
ORACLE_EXPORT int oracle_pair_dists(const double* x, int64_t n, int64_t L, double flat_eps,
                                    const int64_t* pairs, int64_t m, double* out) {
  int64_t N = n - L + 1;
  if (L < 2 || N < 1) return -1;
  double* mu = (double*)malloc(sizeof(double) * N);
  double* sg = (double*)malloc(sizeof(double) * N);
  uint8_t* fl = (uint8_t*)malloc(N);
  oracle_stats(x, n, L, flat_eps, mu, sg, fl);
  for (int64_t r = 0; r < m; r++) {
    int64_t i = pairs[2 * r], j = pairs[2 * r + 1];
    if (i < 0 || j < 0 || i >= N || j >= N)
      out[r] = NAN;
    else if (fl[i] || fl[j])
      out[r] = INFINITY;
    else
      out[r] = sqrt(sqdist(x, L, i, j, mu, sg));
  }
  free(mu);
  free(sg);
  free(fl);
  return 0;
}

/* Pearson correlation of windows i, j at length L (NaN if either is flat). */
ORACLE_EXPORT double oracle_pearson(const double* x, int64_t n, int64_t L, int64_t i, int64_t j,
                                    double flat_eps) {
  int64_t N = n - L + 1;
  if (i < 0 || j < 0 || i >= N || j >= N) return NAN;
  double* mu = (double*)malloc(sizeof(double) * N);
  double* sg = (double*)malloc(sizeof(double) * N);
  uint8_t* fl = (uint8_t*)malloc(N);
  oracle_stats(x, n, L, flat_eps, mu, sg, fl);
  double r = (fl[i] || fl[j]) ? NAN : pearson(x, L, i, j, mu, sg);
  free(mu);
  free(sg);
  free(fl);
  return r;
}

/* Decision logic of Alg. ComputeSubMP for given per-profile (minDist, maxLB):
 * a profile is valid iff minDist < maxLB; minDistAbs is the smallest minDist of
 * the valid profiles, minLbAbs the smallest maxLB of the non-valid ones, and
 * the motif is certified (bBestM) iff minDistAbs < minLbAbs. */
ORACLE_EXPORT int oracle_submp_decide(int64_t count, const double* minDist, const double* maxLB,
                                      uint8_t* valid, double* minDistAbs, double* minLbAbs) {
  double md = INFINITY, ml = INFINITY;
  for (int64_t i = 0; i < count; i++) {
    if (minDist[i] < maxLB[i]) {
      valid[i] = 1;
      if (minDist[i] < md) md = minDist[i];
    } else {
      valid[i] = 0;
      if (maxLB[i] < ml) ml = maxLB[i];
    }
  }
  *minDistAbs = md;
  *minLbAbs = ml;
  return md < ml ? 1 : 0;
}

/* ---------------------------------------------------------------- rankings */

typedef struct {
  double d;
  int64_t a, b, i, L;
} cand_t;

static int cmp_motif(const void* p, const void* q) {
  const cand_t* u = (const cand_t*)p;
  const cand_t* v = (const cand_t*)q;
  if (u->d != v->d) return u->d < v->d ? -1 : 1;
  if (u->a != v->a) return u->a < v->a ? -1 : 1;
  if (u->b != v->b) return u->b < v->b ? -1 : 1;
  return 0;
}

static int cmp_discord(const void* p, const void* q) {
  const cand_t* u = (const cand_t*)p;
  const cand_t* v = (const cand_t*)q;
  if (u->d != v->d) return u->d > v->d ? -1 : 1;
  if (u->i != v->i) return u->i < v->i ? -1 : 1;
  return 0;
}

static int cmp_gmotif(const void* p, const void* q) {
  const cand_t* u = (const cand_t*)p;
  const cand_t* v = (const cand_t*)q;
  if (u->d != v->d) return u->d < v->d ? -1 : 1;
  if (u->L != v->L) return u->L < v->L ? -1 : 1;
  if (u->i != v->i) return u->i < v->i ? -1 : 1;
  return 0;
}

static int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

/* Top-k motif pairs of one length from its matrix profile. Output rows of
 * (a, b) in mot_ab[2k] and d in mot_d[k]; unused slots -1 / NaN. */
static void topk_motifs(const double* mp, const int64_t* ip, int64_t N, int64_t e, int64_t k,
                        int64_t* mot_ab, double* mot_d) {
  cand_t* c = (cand_t*)malloc(sizeof(cand_t) * (N > 0 ? N : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < N; i++) {
    if (ip[i] < 0 || !isfinite(mp[i])) continue;
    c[m].d = mp[i];
    c[m].a = i < ip[i] ? i : ip[i];
    c[m].b = i < ip[i] ? ip[i] : i;
    c[m].i = i;
    m++;
  }
  qsort(c, m, sizeof(cand_t), cmp_motif);
  int64_t got = 0;
  for (int64_t r = 0; r < m && got < k; r++) {
    int ok = 1;
    for (int64_t s = 0; s < got && ok; s++) {
      int64_t a2 = mot_ab[2 * s], b2 = mot_ab[2 * s + 1];
      if (iabs64(c[r].a - a2) <= e || iabs64(c[r].a - b2) <= e || iabs64(c[r].b - a2) <= e ||
          iabs64(c[r].b - b2) <= e)
        ok = 0;
    }
    if (!ok) continue;
    mot_ab[2 * got] = c[r].a;
    mot_ab[2 * got + 1] = c[r].b;
    mot_d[got] = c[r].d;
    got++;
  }
  for (; got < k; got++) {
    mot_ab[2 * got] = mot_ab[2 * got + 1] = -1;
    mot_d[got] = NAN;
  }
  free(c);
}

/* Top-k 1st discords of one length: (offset, nn) in dis_on[2k], d in dis_d[k]. */
static void topk_discords(const double* mp, const int64_t* ip, int64_t N, int64_t e, int64_t k,
                          int64_t* dis_on, double* dis_d) {
  cand_t* c = (cand_t*)malloc(sizeof(cand_t) * (N > 0 ? N : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < N; i++) {
    if (ip[i] < 0 || !isfinite(mp[i])) continue;
    c[m].d = mp[i];
    c[m].i = i;
    c[m].a = ip[i];
    m++;
  }
  qsort(c, m, sizeof(cand_t), cmp_discord);
  int64_t got = 0;
  for (int64_t r = 0; r < m && got < k; r++) {
    int ok = 1;
    for (int64_t s = 0; s < got && ok; s++)
      if (iabs64(c[r].i - dis_on[2 * s]) <= e) ok = 0;
    if (!ok) continue;
    dis_on[2 * got] = c[r].i;
    dis_on[2 * got + 1] = c[r].a;
    dis_d[got] = c[r].d;
    got++;
  }
  for (; got < k; got++) {
    dis_on[2 * got] = dis_on[2 * got + 1] = -1;
    dis_d[got] = NAN;
  }
  free(c);
}

/*
 * Full variable-length run: for every L in [l_min, l_max], the exact matrix
 * profile (all owners), the VALMP update, top-k motifs and discords; then the
 * cross-length rankings. Output layouts (caller-allocated):
 *   prof_dist[(L-l_min)*N0 + i], prof_idx[...]   N0 = n - l_min + 1; entries
 *       i >= N_L hold +inf / -1
 *   valmp_norm[N0], valmp_dist[N0], valmp_len[N0], valmp_idx[N0]
 *   mot_ab[(L-l_min)*2k_m + 2r + {0,1}], mot_d[(L-l_min)*k_m + r]
 *   dis_on[(L-l_min)*2k_d + 2r + {0,1}], dis_d[(L-l_min)*k_d + r]
 *   g_mot_abl[3k_m] (a, b, L), g_mot_d[2k_m] (d, d/sqrt(L))
 *   g_dis_onl[3k_d] (offset, nn, L), g_dis_d[2k_d] (d, d/sqrt(L))
 */
ORACLE_EXPORT int oracle_valmod(const double* x, int64_t n, int64_t l_min, int64_t l_max,
                                int64_t excl_den, double flat_eps, int64_t k_m, int64_t k_d,
                                int nthreads, double* prof_dist, int64_t* prof_idx,
                                double* valmp_norm, double* valmp_dist, int64_t* valmp_len,
                                int64_t* valmp_idx, int64_t* mot_ab, double* mot_d,
                                int64_t* dis_on, double* dis_d, int64_t* g_mot_abl,
                                double* g_mot_d, int64_t* g_dis_onl, double* g_dis_d) {
  if (l_min < 2 || l_max < l_min || excl_den < 1 || n - l_max + 1 < 1) return -1;
  int64_t N0 = n - l_min + 1;
  int64_t nlen = l_max - l_min + 1;
  for (int64_t i = 0; i < N0; i++) {
    valmp_norm[i] = INFINITY;
    valmp_dist[i] = INFINITY;
    valmp_len[i] = 0;
    valmp_idx[i] = -1;
  }
  for (int64_t t = 0; t < nlen; t++) {
    int64_t L = l_min + t;
    int64_t N = n - L + 1;
    double* dist = prof_dist + t * N0;
    int64_t* idx = prof_idx + t * N0;
    oracle_profile_rows(x, n, L, excl_den, flat_eps, NULL, N, dist, idx, nthreads);
    for (int64_t i = N; i < N0; i++) {
      dist[i] = INFINITY;
      idx[i] = -1;
    }
    /* Alg. updateVALMP: length-normalise by sqrt(1/L), keep the strictly smaller */
    for (int64_t i = 0; i < N; i++) {
      double nd = dist[i] * sqrt(1.0 / (double)L);
      if (nd < valmp_norm[i]) {
        valmp_norm[i] = nd;
        valmp_dist[i] = dist[i];
        valmp_len[i] = L;
        valmp_idx[i] = idx[i];
      }
    }
    int64_t e = excl_zone(L, excl_den);
    topk_motifs(dist, idx, N, e, k_m, mot_ab + t * 2 * k_m, mot_d + t * k_m);
    topk_discords(dist, idx, N, e, k_d, dis_on + t * 2 * k_d, dis_d + t * k_d);
  }
  /* cross-length discords: position-wise max of d / sqrt(L), strict */
  for (int64_t r = 0; r < k_d; r++) {
    double best = -INFINITY;
    g_dis_onl[3 * r] = g_dis_onl[3 * r + 1] = g_dis_onl[3 * r + 2] = -1;
    g_dis_d[2 * r] = g_dis_d[2 * r + 1] = NAN;
    for (int64_t t = 0; t < nlen; t++) {
      double d = dis_d[t * k_d + r];
      if (!(d == d)) continue;
      int64_t L = l_min + t;
      double dn = d / sqrt((double)L);
      if (dn > best) {
        best = dn;
        g_dis_onl[3 * r] = dis_on[t * 2 * k_d + 2 * r];
        g_dis_onl[3 * r + 1] = dis_on[t * 2 * k_d + 2 * r + 1];
        g_dis_onl[3 * r + 2] = L;
        g_dis_d[2 * r] = d;
        g_dis_d[2 * r + 1] = dn;
      }
    }
  }
  /* cross-length motifs from the final VALMP */
  cand_t* c = (cand_t*)malloc(sizeof(cand_t) * N0);
  int64_t m = 0;
  for (int64_t i = 0; i < N0; i++) {
    if (valmp_idx[i] < 0 || !isfinite(valmp_norm[i])) continue;
    c[m].d = valmp_norm[i];
    c[m].L = valmp_len[i];
    c[m].i = i;
    c[m].a = i < valmp_idx[i] ? i : valmp_idx[i];
    c[m].b = i < valmp_idx[i] ? valmp_idx[i] : i;
    m++;
  }
  qsort(c, m, sizeof(cand_t), cmp_gmotif);
  int64_t got = 0;
  for (int64_t r = 0; r < m && got < k_m; r++) {
    int ok = 1;
    for (int64_t s = 0; s < got && ok; s++) {
      int64_t a2 = g_mot_abl[3 * s], b2 = g_mot_abl[3 * s + 1], L2 = g_mot_abl[3 * s + 2];
      int64_t Lm = c[r].L > L2 ? c[r].L : L2;
      int64_t e = excl_zone(Lm, excl_den);
      if (iabs64(c[r].a - a2) <= e || iabs64(c[r].a - b2) <= e || iabs64(c[r].b - a2) <= e ||
          iabs64(c[r].b - b2) <= e)
        ok = 0;
    }
    if (!ok) continue;
    g_mot_abl[3 * got] = c[r].a;
    g_mot_abl[3 * got + 1] = c[r].b;
    g_mot_abl[3 * got + 2] = c[r].L;
    g_mot_d[2 * got] = valmp_dist[c[r].i];
    g_mot_d[2 * got + 1] = c[r].d;
    got++;
  }
  for (; got < k_m; got++) {
    g_mot_abl[3 * got] = g_mot_abl[3 * got + 1] = g_mot_abl[3 * got + 2] = -1;
    g_mot_d[2 * got] = g_mot_d[2 * got + 1] = NAN;
  }
  free(c);
  return 0;
}

/*
 * m-th best matches (Def. m-th best match): the m smallest entries of the
 * distance profile of each listed owner at length L, excluding the owner's
 * trivial matches (the neighbours may be trivial matches of each other), in
 * order of (distance, index); missing entries are +inf / -1. Flat owners have
 * none; flat candidates are skipped. dist[r*m + j], idx[r*m + j].
 */
typedef struct {
  double d;
  int64_t j;
} dj_t;

static int cmp_dj(const void* p, const void* q) {
  const dj_t* u = (const dj_t*)p;
  const dj_t* v = (const dj_t*)q;
  if (u->d != v->d) return u->d < v->d ? -1 : 1;
  return u->j < v->j ? -1 : (u->j > v->j ? 1 : 0);
}

ORACLE_EXPORT int oracle_mth_rows(const double* x, int64_t n, int64_t L, int64_t excl_den, double flat_eps,
                                  int64_t m, const int64_t* rows, int64_t nrows, double* dist, int64_t* idx) {
  int64_t N = n - L + 1;
  if (L < 2 || N < 1 || excl_den < 1 || m < 1) return -1;
  double* mu = (double*)malloc(sizeof(double) * N);
  double* sg = (double*)malloc(sizeof(double) * N);
  uint8_t* fl = (uint8_t*)malloc(N);
  dj_t* prof = (dj_t*)malloc(sizeof(dj_t) * N);
  oracle_stats(x, n, L, flat_eps, mu, sg, fl);
  int64_t e = excl_zone(L, excl_den);
  int64_t cnt = rows ? nrows : N;
  for (int64_t r = 0; r < cnt; r++) {
    int64_t i = rows ? rows[r] : r;
    int64_t got = 0;
    if (i >= 0 && i < N && !fl[i]) {
      for (int64_t j = 0; j < N; j++) {
        if (fl[j] || iabs64(i - j) <= e) continue;
        prof[got].d = sqrt(sqdist(x, L, i, j, mu, sg));
        prof[got].j = j;
        got++;
      }
      qsort(prof, got, sizeof(dj_t), cmp_dj);
    }
    for (int64_t q = 0; q < m; q++) {
      dist[r * m + q] = q < got ? prof[q].d : INFINITY;
      idx[r * m + q] = q < got ? prof[q].j : -1;
    }
  }
  free(mu);
  free(sg);
  free(fl);
  free(prof);
  return 0;
}

/*
 * Top-k m-th discords (Defs. m-th discord and Top-k m-th discord), for every
 * j = 1..m and length L: owners by their j-th best-match distance, descending
 * (ties to the smaller offset), accepted greedily unless within the exclusion
 * zone of an owner already accepted for the same j (the rule of the 1st
 * discords); owners with fewer than j candidates are skipped. Across lengths
 * (Alg. UpdateVariableLengthDiscords): for each (j, rank) the largest d / sqrt(L),
 * strictly (the shorter length keeps ties).
 *   on[((t*m + j)*k + r)*2 + {0,1}] (offset, j-th neighbour), d[(t*m + j)*k + r]
 *   g_onl[((j*k) + r)*3 + {0,1,2}] (offset, neighbour, L), g_d[(j*k + r)*2 + {0,1}] (d, d/sqrt(L))
 */
ORACLE_EXPORT int oracle_mth_discords(const double* x, int64_t n, int64_t l_min, int64_t l_max, int64_t excl_den,
                                      double flat_eps, int64_t k, int64_t m, int64_t* on, double* d,
                                      int64_t* g_onl, double* g_d) {
  if (l_min < 2 || l_max < l_min || excl_den < 1 || k < 1 || m < 1 || n - l_max + 1 < 1) return -1;
  int64_t nlen = l_max - l_min + 1;
  for (int64_t t = 0; t < nlen; t++) {
    int64_t L = l_min + t;
    int64_t N = n - L + 1;
    int64_t e = excl_zone(L, excl_den);
    double* md = (double*)malloc(sizeof(double) * N * m);
    int64_t* mi = (int64_t*)malloc(sizeof(int64_t) * N * m);
    double* col = (double*)malloc(sizeof(double) * N);
    int64_t* nn = (int64_t*)malloc(sizeof(int64_t) * N);
    oracle_mth_rows(x, n, L, excl_den, flat_eps, m, NULL, N, md, mi);
    for (int64_t j = 0; j < m; j++) {
      for (int64_t i = 0; i < N; i++) {
        col[i] = md[i * m + j];
        nn[i] = mi[i * m + j];
      }
      topk_discords(col, nn, N, e, k, on + (t * m + j) * k * 2, d + (t * m + j) * k);
    }
    free(md);
    free(mi);
    free(col);
    free(nn);
  }
  for (int64_t j = 0; j < m; j++)
    for (int64_t r = 0; r < k; r++) {
      int64_t* go = g_onl + (j * k + r) * 3;
      double* gd = g_d + (j * k + r) * 2;
      go[0] = go[1] = go[2] = -1;
      gd[0] = gd[1] = NAN;
      double best = -INFINITY;
      for (int64_t t = 0; t < nlen; t++) {
        double v = d[(t * m + j) * k + r];
        if (!(v == v)) continue;
        int64_t L = l_min + t;
        double dn = v / sqrt((double)L);
        if (dn > best) {
          best = dn;
          go[0] = on[((t * m + j) * k + r) * 2];
          go[1] = on[((t * m + j) * k + r) * 2 + 1];
          go[2] = L;
          gd[0] = v;
          gd[1] = dn;
        }
      }
    }
  return 0;
}

/*
 * Variable-length motif sets (Def. data series motif set; Problem of
 * variable-length motif sets discovery; Sec. "Finding Motif Sets"): for each
 * given motif pair (a, b) of length L and distance d, in the given order, the
 * radius is r = D * d and the candidate members are the windows of length L at
 * distance < r from a or from b (each with its distance to the nearer of the
 * two). Members are taken in order of (that distance, offset); a candidate is
 * dropped if its offset already belongs to an earlier set (the sets are
 * disjoint by offset) or if it lies within the exclusion zone of a member
 * already taken for this set (trivial matches removed). Flat windows are never
 * members. Outputs per set s: count[s] (members), and the first `cap` members
 * off[s*cap + i] / dist[s*cap + i] (-1 / NaN after the last).
 */
typedef struct {
  double d;
  int64_t c;
} mem_t;

static int cmp_mem(const void* p, const void* q) {
  const mem_t* u = (const mem_t*)p;
  const mem_t* v = (const mem_t*)q;
  if (u->d != v->d) return u->d < v->d ? -1 : 1;
  return u->c < v->c ? -1 : (u->c > v->c ? 1 : 0);
}

ORACLE_EXPORT int oracle_motif_sets(const double* x, int64_t n, int64_t k, const int64_t* pairs_abl,
                                    const double* pair_d, double D, int64_t excl_den, double flat_eps, int64_t cap,
                                    int64_t* count, int64_t* off, double* dist) {
  if (k < 0 || cap < 1 || excl_den < 1 || !(D >= 0.0)) return -1;
  uint8_t* taken = (uint8_t*)calloc((size_t)n, 1);
  for (int64_t s = 0; s < k; s++) {
    const int64_t a = pairs_abl[3 * s], b = pairs_abl[3 * s + 1], L = pairs_abl[3 * s + 2];
    count[s] = 0;
    for (int64_t i = 0; i < cap; i++) {
      off[s * cap + i] = -1;
      dist[s * cap + i] = NAN;
    }
    if (a < 0 || L < 2 || n - L + 1 < 1) continue;
    const int64_t N = n - L + 1;
    const double r = D * pair_d[s];
    double* mu = (double*)malloc(sizeof(double) * N);
    double* sg = (double*)malloc(sizeof(double) * N);
    uint8_t* fl = (uint8_t*)malloc(N);
    oracle_stats(x, n, L, flat_eps, mu, sg, fl);
    mem_t* m = (mem_t*)malloc(sizeof(mem_t) * N);
    int64_t cnt = 0;
    for (int64_t c = 0; c < N; c++) {
      if (fl[c]) continue;
      double best = INFINITY;
      if (!fl[a]) best = sqrt(sqdist(x, L, a, c, mu, sg));
      if (!fl[b]) {
        double db = sqrt(sqdist(x, L, b, c, mu, sg));
        if (db < best) best = db;
      }
      if (best < r) {
        m[cnt].d = best;
        m[cnt].c = c;
        cnt++;
      }
    }
    qsort(m, cnt, sizeof(mem_t), cmp_mem);
    const int64_t e = excl_zone(L, excl_den);
    int64_t got = 0;
    int64_t* acc = (int64_t*)malloc(sizeof(int64_t) * (cnt > 0 ? cnt : 1));
    for (int64_t q = 0; q < cnt; q++) {
      const int64_t c = m[q].c;
      if (taken[c]) continue;
      int ok = 1;
      for (int64_t u = 0; u < got && ok; u++)
        if (iabs64(c - acc[u]) <= e) ok = 0;
      if (!ok) continue;
      acc[got] = c;
      if (got < cap) {
        off[s * cap + got] = c;
        dist[s * cap + got] = m[q].d;
      }
      got++;
    }
    for (int64_t u = 0; u < got; u++) taken[acc[u]] = 1;
    count[s] = got;
    free(acc);
    free(m);
    free(mu);
    free(sg);
    free(fl);
  }
  free(taken);
  return 0;
}

/*
 * Valid fraction of the lower-bound test at length L for partial distance
 * profiles built at base length b (Alg. ComputeMatrixProfile heaps, Alg.
 * ComputeSubMP test), used for diagnostics. Heap of owner o: the p candidates
 * with the largest correlation at b (ties to the smaller index; equivalently the
 * p smallest lower bounds). The bound for every candidate not stored uses the
 * largest correlation among them (the (p+1)-th overall, clamped at 0; no such
 * candidate: +inf bound). Windows flat at b are not stored; each one that is a
 * candidate at L (non-flat, non-trivial) contributes its own bound, from its
 * real correlation at b (0 only for an exactly constant window), and the bound
 * of the owner is the smallest of these. Valid iff the smallest exact distance at L among the
 * stored candidates that are still eligible at L is strictly below that bound.
 * valid_out[o] is 1/0 for owners o < N_L that are non-flat at L, 2 otherwise.
 */
typedef struct {
  double r;
  int64_t c;
} rc_t;

static int cmp_rc(const void* p, const void* q) {
  const rc_t* u = (const rc_t*)p;
  const rc_t* v = (const rc_t*)q;
  if (u->r != v->r) return u->r > v->r ? -1 : 1;
  return u->c < v->c ? -1 : (u->c > v->c ? 1 : 0);
}

ORACLE_EXPORT int64_t oracle_valid_fraction(const double* x, int64_t n, int64_t b, int64_t L,
                                            int64_t p, int64_t excl_den, double flat_eps,
                                            uint8_t* valid_out) {
  int64_t Nb = n - b + 1, NL = n - L + 1;
  if (L < b || NL < 1 || p < 1) return -1;
  double *mub = malloc(sizeof(double) * Nb), *sgb = malloc(sizeof(double) * Nb);
  uint8_t* flb = malloc(Nb);
  double *muL = malloc(sizeof(double) * NL), *sgL = malloc(sizeof(double) * NL);
  uint8_t* flL = malloc(NL);
  oracle_stats(x, n, b, flat_eps, mub, sgb, flb);
  oracle_stats(x, n, L, flat_eps, muL, sgL, flL);
  int64_t eb = excl_zone(b, excl_den), eL = excl_zone(L, excl_den);
  rc_t* list = malloc(sizeof(rc_t) * Nb);
  int64_t nvalid = 0;
  for (int64_t o = 0; o < NL; o++) {
    if (flL[o]) {
      valid_out[o] = 2;
      continue;
    }
    if (flb[o]) { /* lower bound 0: never valid */
      valid_out[o] = 0;
      continue;
    }
    int64_t m = 0;
    double flat_lb = INFINITY;
    for (int64_t c = 0; c < Nb; c++) {
      if (iabs64(c - o) <= eb) continue;
      if (flb[c]) {
        /* never stored; its own bound (with its real base correlation) joins the
         * bound of the candidates not stored when it is a candidate at L */
        if (c < NL && !flL[c] && iabs64(c - o) > eL) {
          double q = sgb[c] > 0.0 ? pearson(x, b, o, c, mub, sgb) : 0.0;
          if (q < 0.0) q = 0.0;
          double base = 1.0 - q * q;
          if (base < 0.0) base = 0.0;
          double lbc = sqrt((double)b * base) * sgb[o] / sgL[o];
          if (lbc < flat_lb) flat_lb = lbc;
        }
        continue;
      }
      list[m].r = pearson(x, b, o, c, mub, sgb);
      list[m].c = c;
      m++;
    }
    qsort(list, m, sizeof(rc_t), cmp_rc);
    int64_t stored = m < p ? m : p;
    double bound = flat_lb;
    if (m > p) {
      double q = list[p].r;
      if (q < 0.0) q = 0.0;
      double base = 1.0 - q * q;
      if (base < 0.0) base = 0.0;
      double lbn = sqrt((double)b * base) * sgb[o] / sgL[o];
      if (lbn < bound) bound = lbn;
    }
    double md = INFINITY;
    for (int64_t s = 0; s < stored; s++) {
      int64_t c = list[s].c;
      if (c >= NL || iabs64(c - o) <= eL || flL[c]) continue;
      double d = sqrt(sqdist(x, L, o, c, muL, sgL));
      if (d < md) md = d;
    }
    valid_out[o] = md < bound ? 1 : 0;
    nvalid += valid_out[o];
  }
  free(list);
  free(mub);
  free(sgb);
  free(flb);
  free(muL);
  free(sgL);
  free(flL);
  return nvalid;
}
