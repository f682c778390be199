// C ABI of the VALMOD library: plan validation, workspace layout and the
// per-length driver (Alg. VALMOD) that enqueues the kernels.
#include "../../include/valmod.h"
#include "valmod_common.h"
#include "valmod_kernels.h"

#include <algorithm>
#include <chrono>
#include <math.h>
#include <mutex>
#include <new>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

using namespace valmod;

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kRingRows = 32;  // profile rows kept in the workspace (rankings run per group of rows)
// a lane's pinned host words: 0-5 NFAIL .. MINLB and 6 MOPEN after a sweep, then
constexpr int kErrSlot = 7;   // the device error flag
constexpr int kOverSlot = 8;  // the last rebuild's overflowing lists (CNT_OVER)
constexpr int kHostWords = 16;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct WsLayout {
  size_t xs, A, B, A2, B2, mu, sig, invn, flat, df, dg, sw32, thr, thr32, best, counters, anc;
  size_t hc, hS, hn, hbound, hsig, hflat, acnt, abuf, fail, big, lbm, rec, part, mvals, mnn, mkeys;
  size_t mstate, mub, mlist, tau_on, tau_d;
  size_t thrp;  // thresholds of a rebuild from the partial profiles it replaces
  size_t df32, dg32, inv32, bsw_max, bsw_min, bdf_max, bdg_max, bmu_max, delta64, delta, hard;
  size_t ms_keys0, ms_keys1, ms_vals0, ms_vals1, ms_hist, ms_meta, ms_count, ms_taken, ms_bucket;
  // the last ring_rows profile rows (distance, index; stride N0 of the series):
  // seeds of the next length and input of the per-length rankings
  size_t ring_d, ring_i;
  int64_t ring_rows;
  // stand-ins for outputs the caller skips but the run reads back
  size_t sub_vn, sub_vd, sub_vl, sub_vi, sub_mab, sub_md, sub_don, sub_dd, sub_gab, sub_gd, sub_gdon, sub_gdd;
  size_t total;
};

// Geometry of the diagonal pass of one series, fixed for all its lengths.
struct PassGeom {
  int64_t dstart = 0, H = 0, segs = 0, bands = 0, stride = 0;
  int K = 0;
  bool table = true;  // FP64 anchor table (FP64 recurrence); FP32 items compute their anchors directly
};

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v && *v ? atoi(v) : dflt;
}

PassGeom pass_geom(int64_t n, int32_t l_min, int32_t excl_den, bool fp32, int32_t refresh_R, int hmul, int kdiag) {
  PassGeom g;
  const int64_t N0 = n - l_min + 1;
  const int64_t e0 = excl_zone(l_min, excl_den);
  g.K = kdiag == 4 || kdiag == 8 ? kdiag : (env_int(fp32 ? "VALMOD_PASS_K32" : "VALMOD_PASS_K", 8) == 4 ? 4 : 8);
  const int64_t bw = 64 * g.K;
  g.dstart = (e0 + 1) / 8 * 8;  // bands start on a multiple of 8 (aligned wide loads)
  g.bands = (N0 - g.dstart + bw - 1) / bw;
  g.stride = g.bands * bw;
  // FP64 anchor table (one anchor per segment start and diagonal, grown by one
  // term per length) while it fits this budget; beyond it anchors are formed directly
  const double budget = (double)env_int("VALMOD_ANCHOR_BUDGET_MIB", 32768) * 1048576.0;
  auto table_bytes = [&](int64_t H) { return (double)((N0 - g.dstart + H - 1) / H) * (double)g.stride * 8.0; };
  int64_t H;
  if (fp32) {
    // FP32 recurrence: segments of R rows restart from FP64 anchors (the refresh
    // interval); the rounding bound grows linearly with R
    H = refresh_R;
    if (H <= 0) {
      H = 256;
      while (H < 1024 && table_bytes(H) > budget) H *= 2;
    }
  } else {
    const int64_t ndiag = N0 - 1 - e0;
    const double cells = ndiag > 0 ? 0.5 * (double)ndiag * (double)(ndiag + 1) : 0.0;
    // segment height: enough work items to keep every SIMD busy, within [128, 4096]
    const double items = env_int("VALMOD_PASS_ITEMS", 16384);
    H = 4096;
    while (H > 128 && cells / ((double)bw * (double)H) < items) H /= 2;
    H *= hmul;  // autotuned: taller segments trade work items for per-item overhead
    if (H > 8192) H = 8192;
    const int hforce = env_int("VALMOD_PASS_H", 0);
    if (hforce >= 64 && hforce % 8 == 0) H = hforce;
  }
  g.H = H;
  g.segs = (N0 - g.dstart + H - 1) / H;
  g.table = table_bytes(H) <= budget;
  return g;
}

}  // namespace

// --------------------------------------------------------------------------
// Static scratch of valmod_run_noalloc: the workspace of a plan that needs at
// most VALMOD_NOALLOC_SCRATCH_BYTES lives in this array instead of a caller
// buffer. Every GPU the library runs on holds its own copy until the process
// ends; its device address is taken once per device (with that device current)
// and kept, since the array's name is only a host-side stand-in.
static __device__ __align__(256) unsigned char scratch[VALMOD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// device address of `scratch` on device `dev`, which must be current
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

// A lane runs its series one after another on its own stream; lanes run
// concurrently.
struct Lane {
  std::vector<int> series;  // assigned series, in run order
  size_t base = 0;          // byte offset of the lane's workspace
  WsLayout ws;              // offsets relative to base
  int64_t nmax = 0, n0max = 0, ancmax = 0, itemmax = 0, total_lengths = 0, nlenmax = 0;
  double cost = 0.0;
  // device resources (created on the plan's device at the first run)
  hipStream_t st = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
  unsigned long long* hcnt = nullptr;  // pinned host copy of a few counters
  std::vector<hipEvent_t> ev;         // pass timing
  int64_t nev = 0;                     // events recorded by the last run
};

struct valmod_plan_s {
  valmod_config cfg;
  std::vector<int64_t> n;
  std::vector<int32_t> lmin, lmax;
  std::vector<valmod_layout> lay;
  valmod_sizes sizes;
  int64_t cap = 0;  // candidate-list capacity per owner of the collecting pass
  std::vector<PassGeom> geom;
  std::vector<Lane> lanes;
  size_t ws_total = 0;
  int res_device = -1;
  hipEvent_t start = nullptr, g0 = nullptr, g1 = nullptr;
  // captured run (graph mode), valid for one set of buffers and one stream
  hipGraphExec_t exec = nullptr;
  const void* key_series = nullptr;
  void* key_ws = nullptr;
  hipStream_t key_stream = nullptr;
  valmod_outputs key_out;
  int64_t graph_cells = 0;
  hipEvent_t finished = nullptr;  // end of the last enqueued run (after its error-flag copies)
  bool run_pending = false;       // a run was enqueued and valmod_run_status has not read it yet
  // the last run was valmod_run_noalloc's: its scratch address and stream
  bool na_pending = false;
  char* na_ws = nullptr;
  hipStream_t na_stream = nullptr;
  valmod_status last_status = VALMOD_OK;
  // autotuned geometry: FP64 segment-height multiplier, FP32 refresh interval (0: default)
  int tune_hmul = 1;
  int32_t tune_R = 0;
  int tune_K = 0;  // diagonals per lane (0: default)
  bool tune_no_heaps = false;  // the autotuner found that partial profiles do not pay
  double pass_ms = 0.0;
  int64_t pass_launches = 0, pass_cells = 0;
};

static valmod_status fail(valmod_status s) { return s; }

extern "C" const char* valmod_status_str(int status) {
  switch (status) {
    case VALMOD_OK: return "ok";
    case VALMOD_E_ARG: return "invalid argument";
    case VALMOD_E_TOO_SHORT: return "series too short for the length range";
    case VALMOD_E_NOMEM: return "host allocation failed";
    case VALMOD_E_HIP: return "HIP runtime error";
    case VALMOD_E_LAYOUT: return "sizes exceed the supported index range";
    case VALMOD_E_DEVICE: return "device-side error (non-finite input or capacity exceeded)";
    case VALMOD_E_SCRATCH: return "the plan's workspace exceeds the static scratch of valmod_run_noalloc";
    default: return "unknown status";
  }
}

// workspace of one lane, sized for the largest of its series
static size_t layout_lane(const valmod_plan_s* P, Lane& ln) {
  WsLayout& w = ln.ws;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t np = (size_t)(ln.nmax + kPad);
  const size_t wp = (size_t)(ln.n0max + kPad);
  w.xs = take(np * 8);
  w.A = take(wp * 8);
  w.B = take(wp * 8);
  w.A2 = take(wp * 8);  // the anchored sums alternate between two buffers by length
  w.B2 = take(wp * 8);
  w.mu = take(wp * 8);
  w.sig = take(wp * 8);
  w.invn = take(wp * 8);
  w.flat = take(wp);
  w.df = take(wp * 8);
  w.dg = take(wp * 8);
  w.sw32 = take(wp * 4);
  w.thr = take(wp * 8);
  w.thr32 = take(wp * 4);
  w.best = take(wp * 8);
  w.counters = take(CNT_WORDS * 8);
  w.anc = take((size_t)ln.ancmax * 8);
  const size_t pp = (size_t)P->cfg.p;
  w.hc = take(wp * pp * 4);
  w.hS = take(wp * pp * 8);
  w.hn = take(wp * 4);
  w.hbound = take(wp * 8);
  w.hsig = take(wp * 8);
  w.hflat = take(wp);
  w.thrp = take(wp * 8);
  w.acnt = take(wp * 4);
  w.abuf = take((size_t)ln.n0max * (size_t)P->cap * 4);
  w.fail = take(wp * 4);
  w.big = take(wp * 4);
  if (P->cfg.m_discords > 1) {
    const size_t md = (size_t)P->cfg.m_discords;
    w.mvals = take(md * wp * 8);
    w.mnn = take(md * wp * 4);
    w.mkeys = take(md * wp * 8);
    const size_t kdd = (size_t)P->cfg.k_discords;
    w.mstate = take(wp);
    w.mub = take(md * wp * 8);
    w.mlist = take(wp * 4);
    w.tau_on = take(md * kdd * 2 * 4);
    w.tau_d = take(md * kdd * 8);
  }
  if (P->cfg.mset_radius > 0.0) {
    const size_t cc = (size_t)P->cfg.k_motifs * (size_t)ln.n0max;
    w.ms_keys0 = take(cc * 8);
    w.ms_keys1 = take(cc * 8);
    w.ms_vals0 = take(cc * 8);
    w.ms_vals1 = take(cc * 8);
    w.ms_hist = take(motif_sets_hist_words((int64_t)cc) * 4);
    w.ms_meta = take(5 * 64 * 8);
    w.ms_count = take(65 * 4);
    w.ms_taken = take(((size_t)ln.n0max + 63) / 64 * 8);
    w.ms_bucket = take(((size_t)ln.n0max / 2 + 2) * 4);
  }
  if (P->cfg.mode == VALMOD_MODE_PAPER) {
    w.lbm = take(wp * 8);
    w.rec = take(wp * 4);
    w.part = take(wp * 4);
  }
  // per-64-window extrema and per-item rounding bounds of the recurrence (both precisions)
  const size_t nb = wp / 64 + 2;
  w.bsw_max = take(nb * 4);
  w.bsw_min = take(nb * 4);
  w.bdf_max = take(nb * 4);
  w.bdg_max = take(nb * 4);
  w.bmu_max = take(nb * 4);
  w.delta64 = take((size_t)ln.itemmax * 4);
  if (P->cfg.precision == VALMOD_PREC_FP32_REFRESH) {
    w.df32 = take(wp * 4);
    w.dg32 = take(wp * 4);
    w.inv32 = take(wp * 4);
    w.delta = take((size_t)ln.itemmax * 4);
    w.hard = take((size_t)ln.itemmax * 4);
  }
  w.ring_rows = std::min<int64_t>(ln.nlenmax, kRingRows);
  w.ring_d = take((size_t)(w.ring_rows * ln.n0max + kPad) * 8);
  w.ring_i = take((size_t)(w.ring_rows * ln.n0max + kPad) * 4);
  const size_t km = (size_t)P->cfg.k_motifs, kd = (size_t)P->cfg.k_discords, nl = (size_t)ln.nlenmax;
  w.sub_vn = take(wp * 8);
  w.sub_vd = take(wp * 8);
  w.sub_vl = take(wp * 4);
  w.sub_vi = take(wp * 4);
  w.sub_mab = take(nl * km * 2 * 4);
  w.sub_md = take(nl * km * 8);
  w.sub_don = take(nl * kd * 2 * 4);
  w.sub_dd = take(nl * kd * 8);
  w.sub_gab = take(km * 3 * 4);
  w.sub_gd = take(km * 2 * 8);
  w.sub_gdon = take(kd * 3 * 4);
  w.sub_gdd = take(kd * 2 * 8);
  w.total = off;
  return off;
}

// pass geometry of every series and the workspace of every lane (the lane
// assignment is fixed at plan time)
static void build_layout(valmod_plan_s* P) {
  const bool fp32 = P->cfg.precision == VALMOD_PREC_FP32_REFRESH;
  const int32_t R = P->cfg.refresh_R > 0 ? P->cfg.refresh_R : P->tune_R;
  P->geom.clear();
  for (int s = 0; s < P->cfg.num_series; ++s)
    P->geom.push_back(pass_geom(P->n[s], P->lmin[s], P->cfg.excl_den, fp32, R, P->tune_hmul, P->tune_K));
  size_t off = 0;
  for (Lane& ln : P->lanes) {
    ln.nmax = ln.n0max = ln.ancmax = ln.itemmax = ln.total_lengths = 0;
    for (int s : ln.series) {
      const PassGeom& gg = P->geom[s];
      ln.nmax = std::max(ln.nmax, P->n[s]);
      ln.n0max = std::max(ln.n0max, P->lay[s].n0);
      if (gg.table) ln.ancmax = std::max(ln.ancmax, gg.segs * gg.stride);
      ln.itemmax = std::max(ln.itemmax, gg.segs * gg.bands);
      ln.total_lengths += P->lay[s].nlen;
      ln.nlenmax = std::max(ln.nlenmax, P->lay[s].nlen);
    }
    ln.base = off;
    off += align_up(layout_lane(P, ln));
  }
  P->ws_total = off;
}

extern "C" valmod_status valmod_plan(const valmod_config* cfg, valmod_plan_t* out) {
  if (!cfg || !out) return fail(VALMOD_E_ARG);
  *out = nullptr;
  if (cfg->num_series < 1 || !cfg->n || !cfg->l_min || !cfg->l_max) return fail(VALMOD_E_ARG);
  if (cfg->p < 0 || cfg->k_motifs < 1 || cfg->k_discords < 1 || cfg->k_motifs > 64 || cfg->k_discords > 64)
    return fail(VALMOD_E_ARG);
  if (cfg->excl_den < 0 || !(cfg->flat_eps >= 0.0)) return fail(VALMOD_E_ARG);
  if (cfg->refresh_R != 0 && (cfg->refresh_R < 64 || cfg->refresh_R > 8192 || cfg->refresh_R % 16))
    return fail(VALMOD_E_ARG);
  if (cfg->dtype != VALMOD_F32 && cfg->dtype != VALMOD_F64) return fail(VALMOD_E_ARG);
  if (cfg->precision != VALMOD_PREC_FP64 && cfg->precision != VALMOD_PREC_FP32_REFRESH)
    return fail(VALMOD_E_ARG);
  if (cfg->path < VALMOD_PATH_AUTO || cfg->path > VALMOD_PATH_RECOMPUTE || cfg->device < 0)
    return fail(VALMOD_E_ARG);
  if (cfg->lanes < 0 || cfg->lanes > 64 || (cfg->graph != 0 && cfg->graph != 1)) return fail(VALMOD_E_ARG);
  // a captured run takes no host decisions: partial profiles (which need them) are off
  if (cfg->graph && cfg->path == VALMOD_PATH_RECOMPUTE) return fail(VALMOD_E_ARG);
  // capture of the FP32 path is not supported
  if (cfg->graph && cfg->precision == VALMOD_PREC_FP32_REFRESH) return fail(VALMOD_E_ARG);
  if (cfg->mode != VALMOD_MODE_EXACT && cfg->mode != VALMOD_MODE_PAPER) return fail(VALMOD_E_ARG);
  if (cfg->m_discords < 0 || cfg->m_discords > 16) return fail(VALMOD_E_ARG);
  if (cfg->m_discords > 1 && (cfg->mode != VALMOD_MODE_EXACT || cfg->graph)) return fail(VALMOD_E_ARG);
  if (cfg->mode == VALMOD_MODE_PAPER && (cfg->path != VALMOD_PATH_AUTO || cfg->graph)) return fail(VALMOD_E_ARG);
  if (!(cfg->mset_radius >= 0.0) || cfg->mset_radius > 1e6) return fail(VALMOD_E_ARG);
  if (cfg->mset_radius > 0.0 && (cfg->mset_cap < 1 || cfg->mset_cap > (1 << 20))) return fail(VALMOD_E_ARG);

  valmod_plan_s* P = new (std::nothrow) valmod_plan_s();
  if (!P) return fail(VALMOD_E_NOMEM);
  P->cfg = *cfg;
  if (P->cfg.p == 0) P->cfg.p = 10;
  if (P->cfg.excl_den == 0) P->cfg.excl_den = 4;
  if (P->cfg.flat_eps == 0.0) P->cfg.flat_eps = 1.0 / 1048576.0;
  if (P->cfg.graph) P->cfg.path = VALMOD_PATH_FULL;
  if (P->cfg.m_discords < 1) P->cfg.m_discords = 1;
  if (P->cfg.m_discords > P->cfg.p) {
    delete P;
    return fail(VALMOD_E_ARG);
  }
  const int64_t md = P->cfg.m_discords;
  const int S = cfg->num_series;
  try {
    P->n.assign(cfg->n, cfg->n + S);
    P->lmin.assign(cfg->l_min, cfg->l_min + S);
    P->lmax.assign(cfg->l_max, cfg->l_max + S);
    P->lay.resize(S);
  } catch (...) {
    delete P;
    return fail(VALMOD_E_NOMEM);
  }
  P->cfg.n = nullptr;
  P->cfg.l_min = nullptr;
  P->cfg.l_max = nullptr;

  valmod_sizes& z = P->sizes;
  memset(&z, 0, sizeof(z));
  const int64_t km = P->cfg.k_motifs, kd = P->cfg.k_discords;
  std::vector<double> cost(S, 0.0);
  for (int s = 0; s < S; ++s) {
    const int64_t n = P->n[s];
    const int32_t lo = P->lmin[s], hi = P->lmax[s];
    if (lo < 4 || hi < lo || n < 1) {
      delete P;
      return fail(VALMOD_E_ARG);
    }
    const int64_t e = excl_zone(hi, P->cfg.excl_den);
    if (n - hi + 1 <= e + 1) {
      delete P;
      return fail(VALMOD_E_TOO_SHORT);
    }
    const int64_t n0 = n - lo + 1;
    if (n0 > VALMOD_MAX_WINDOWS) {
      delete P;
      return fail(VALMOD_E_LAYOUT);
    }
    const int64_t nlen = hi - lo + 1;
    valmod_layout& L = P->lay[s];
    L.series = z.series;
    L.prof = z.prof;
    L.valmp = z.valmp;
    L.motif = z.motif;
    L.discord = z.discord;
    L.g_motif = z.g_motif;
    L.g_discord = z.g_discord;
    L.stats = z.stats;
    L.mdiscord = z.mdiscord;
    L.g_mdiscord = z.g_mdiscord;
    L.mset = z.mset;
    L.n = n;
    L.n0 = n0;
    L.nlen = nlen;
    L.l_min = lo;
    L.l_max = hi;
    z.series += n;
    z.prof += nlen * n0;
    z.valmp += n0;
    z.motif += nlen * km;
    z.discord += nlen * kd;
    z.g_motif += km;
    z.g_discord += kd;
    z.stats += nlen * VALMOD_NSTATS;
    if (md > 1) {
      z.mdiscord += nlen * md * kd;
      z.g_mdiscord += md * kd;
    }
    if (P->cfg.mset_radius > 0.0) z.mset += km * (int64_t)P->cfg.mset_cap;
    for (int64_t Lx = lo; Lx <= hi; ++Lx) cost[s] += (double)(n - Lx + 1) * (double)(n - Lx + 1);
  }
  const size_t pp = (size_t)P->cfg.p;
  P->cap = 8 * (int64_t)pp < 64 ? 64 : (8 * (int64_t)pp > 512 ? 512 : 8 * (int64_t)pp);
  // test hook: a smaller list capacity makes owners overflow into the row recompute
  const int cap_env = env_int("VALMOD_COLLECT_CAP", 0);
  if (cap_env > 0) P->cap = cap_env < 512 ? cap_env : 512;

  // lanes: longest-processing-time assignment of the series by sum over lengths of N_L^2
  // default 16 lanes: more streams than hardware queues still overlap the short
  // per-length kernels of one series with the passes of others
  const int nl = std::min(S, P->cfg.lanes > 0 ? (int)P->cfg.lanes : 16);
  try {
    P->lanes.resize(nl);
    std::vector<int> order(S);
    for (int s = 0; s < S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int s : order) {
      int best_lane = 0;
      for (int l = 1; l < nl; ++l)
        if (P->lanes[l].cost < P->lanes[best_lane].cost) best_lane = l;
      Lane& ln = P->lanes[best_lane];
      ln.cost += cost[s];
      ln.series.push_back(s);
    }
  } catch (...) {
    delete P;
    return fail(VALMOD_E_NOMEM);
  }
  for (Lane& ln : P->lanes) std::sort(ln.series.begin(), ln.series.end());
  build_layout(P);
  *out = P;
  return VALMOD_OK;
}

extern "C" size_t valmod_workspace_bytes(valmod_plan_t P) { return P ? P->ws_total : 0; }

extern "C" valmod_status valmod_output_sizes(valmod_plan_t P, valmod_sizes* out) {
  if (!P || !out) return VALMOD_E_ARG;
  *out = P->sizes;
  return VALMOD_OK;
}

extern "C" valmod_status valmod_series_layout(valmod_plan_t P, int32_t s, valmod_layout* out) {
  if (!P || !out || s < 0 || s >= P->cfg.num_series) return VALMOD_E_ARG;
  *out = P->lay[s];
  return VALMOD_OK;
}

static void release_resources(valmod_plan_s* P) {
  // a run still in flight writes into the pinned words and records the events
  if (P->run_pending && P->finished) (void)hipEventSynchronize(P->finished);
  P->run_pending = false;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  P->exec = nullptr;
  for (Lane& ln : P->lanes) {
    for (hipEvent_t e : ln.ev) (void)hipEventDestroy(e);
    ln.ev.clear();
    for (hipEvent_t* e : {&ln.ready, &ln.done})
      if (*e) {
        (void)hipEventDestroy(*e);
        *e = nullptr;
      }
    if (ln.st) (void)hipStreamDestroy(ln.st);
    ln.st = nullptr;
    if (ln.hcnt) (void)hipHostFree(ln.hcnt);
    ln.hcnt = nullptr;
  }
  for (hipEvent_t* e : {&P->start, &P->g0, &P->g1, &P->finished})
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  P->res_device = -1;
}

extern "C" void valmod_plan_free(valmod_plan_t P) {
  if (!P) return;
  int prev = -1;
  const bool sw = P->res_device >= 0 && hipGetDevice(&prev) == hipSuccess && hipSetDevice(P->res_device) == hipSuccess;
  release_resources(P);
  if (sw) (void)hipSetDevice(prev);
  delete P;
}

extern "C" valmod_status valmod_last_pass_timing(valmod_plan_t P, double* ms, int64_t* launches,
                                                 int64_t* cells) {
  if (!P) return VALMOD_E_ARG;
  if (ms) *ms = P->pass_ms;
  if (launches) *launches = P->pass_launches;
  if (cells) *cells = P->pass_cells;
  return VALMOD_OK;
}

// streams (default priority), events and pinned counters of every lane
static hipError_t ensure_resources(valmod_plan_s* P) {
  if (P->res_device == P->cfg.device) return hipSuccess;
  release_resources(P);
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
    return e == hipSuccess;
  };
  ok(hipEventCreateWithFlags(&P->start, hipEventDisableTiming));
  ok(hipEventCreate(&P->g0));
  ok(hipEventCreate(&P->g1));
  ok(hipEventCreateWithFlags(&P->finished, hipEventDisableTiming));
  for (Lane& ln : P->lanes) {
    ok(hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking));
    for (hipEvent_t* ev : {&ln.ready, &ln.done}) ok(hipEventCreateWithFlags(ev, hipEventDisableTiming));
    ok(hipHostMalloc((void**)&ln.hcnt, kHostWords * sizeof(unsigned long long), hipHostMallocDefault));
    for (int64_t i = 0; e == hipSuccess && i < 4 * ln.total_lengths; ++i) {
      hipEvent_t ev;
      if (ok(hipEventCreate(&ev))) ln.ev.push_back(ev);
    }
  }
  if (e == hipSuccess) P->res_device = P->cfg.device;
  return e;
}

namespace {

// The per-length driver of one lane (Alg. VALMOD over each of its series).
// advance() enqueues the work of one length and returns; a length whose
// partial-profile sweep needs its counters on the host first returns BLOCKED
// after enqueueing the sweep and the counter copy, and continues once the
// lane's `ready` event has completed.
struct LaneRun {
  enum Status { CONTINUE, BLOCKED, DONE };
  valmod_plan_s* P = nullptr;
  Lane* ln = nullptr;
  const valmod_outputs* o = nullptr;
  const char* d_series = nullptr;
  bool capture = false;
  bool noalloc = false;     // valmod_run_noalloc: the caller's stream, no events, no partial profiles
  hipStream_t run_st = nullptr;  // stream of the lane's work
  hipError_t err = hipSuccess;
  // workspace
  double *xs, *A, *B, *A2, *B2, *mu, *sig, *invn, *df, *dg, *thr, *anc, *hS, *hbound, *hsig, *lbm;
  uint8_t* flat;
  float *sw32, *thr32, *df32, *dg32, *inv32, *bsw_max, *bsw_min, *bdf_max, *bdg_max, *bmu_max, *delta64, *delta;
  uint8_t* hflat;
  double* thrp;
  uint64_t* best;
  unsigned long long* cnt;
  int32_t *hc, *hn, *abuf, *fail, *big, *hard, *rec, *part, *mnn;
  double* mvals;
  uint64_t* mkeys;
  uint8_t* mstate;
  double *mub, *tau_d;
  int32_t *mlist, *tau_on;
  uint32_t* acnt;
  double* ring_d;
  int32_t* ring_i;
  int64_t ring_rows = 1;
  // stand-ins for skipped outputs
  double *sub_vn, *sub_vd, *sub_md, *sub_dd, *sub_gd, *sub_gdd;
  int32_t *sub_vl, *sub_vi, *sub_mab, *sub_don, *sub_gab, *sub_gdon;
  MotifSetLaunch ms{};
  // state
  size_t si = 0;
  bool open = false;
  int L = 0, phase = 0, base = 0;
  int anc_len = 0;  // length the anchor table holds (0: not formed for this series)
  bool heaps_on = false, probe_next = false;
  int64_t evi = 0;

  void init(valmod_plan_s* P_, Lane* ln_, char* ws, const valmod_outputs* o_, const char* series, bool cap) {
    P = P_;
    ln = ln_;
    o = o_;
    d_series = series;
    capture = cap;
    run_st = ln_->st;
    char* b = ws + ln->base;
    const WsLayout& w = ln->ws;
    xs = (double*)(b + w.xs);
    A = (double*)(b + w.A);
    B = (double*)(b + w.B);
    A2 = (double*)(b + w.A2);
    B2 = (double*)(b + w.B2);
    mu = (double*)(b + w.mu);
    sig = (double*)(b + w.sig);
    invn = (double*)(b + w.invn);
    flat = (uint8_t*)(b + w.flat);
    df = (double*)(b + w.df);
    dg = (double*)(b + w.dg);
    sw32 = (float*)(b + w.sw32);
    thr = (double*)(b + w.thr);
    thr32 = (float*)(b + w.thr32);
    anc = (double*)(b + w.anc);
    best = (uint64_t*)(b + w.best);
    cnt = (unsigned long long*)(b + w.counters);
    hc = (int32_t*)(b + w.hc);
    hS = (double*)(b + w.hS);
    hn = (int32_t*)(b + w.hn);
    hbound = (double*)(b + w.hbound);
    hsig = (double*)(b + w.hsig);
    acnt = (uint32_t*)(b + w.acnt);
    abuf = (int32_t*)(b + w.abuf);
    fail = (int32_t*)(b + w.fail);
    big = (int32_t*)(b + w.big);
    const bool mth = P->cfg.m_discords > 1;
    mvals = mth ? (double*)(b + w.mvals) : nullptr;
    mnn = mth ? (int32_t*)(b + w.mnn) : nullptr;
    mkeys = mth ? (uint64_t*)(b + w.mkeys) : nullptr;
    mstate = mth ? (uint8_t*)(b + w.mstate) : nullptr;
    mub = mth ? (double*)(b + w.mub) : nullptr;
    mlist = mth ? (int32_t*)(b + w.mlist) : nullptr;
    tau_on = mth ? (int32_t*)(b + w.tau_on) : nullptr;
    tau_d = mth ? (double*)(b + w.tau_d) : nullptr;
    const bool paper = P->cfg.mode == VALMOD_MODE_PAPER;
    lbm = paper ? (double*)(b + w.lbm) : nullptr;
    rec = paper ? (int32_t*)(b + w.rec) : nullptr;
    part = paper ? (int32_t*)(b + w.part) : nullptr;
    const bool fp32 = P->cfg.precision == VALMOD_PREC_FP32_REFRESH;
    df32 = fp32 ? (float*)(b + w.df32) : nullptr;
    dg32 = fp32 ? (float*)(b + w.dg32) : nullptr;
    inv32 = fp32 ? (float*)(b + w.inv32) : nullptr;
    bsw_max = (float*)(b + w.bsw_max);
    bsw_min = (float*)(b + w.bsw_min);
    bdf_max = (float*)(b + w.bdf_max);
    bdg_max = (float*)(b + w.bdg_max);
    bmu_max = (float*)(b + w.bmu_max);
    delta64 = (float*)(b + w.delta64);
    hflat = (uint8_t*)(b + w.hflat);
    thrp = (double*)(b + w.thrp);
    ring_d = (double*)(b + w.ring_d);
    ring_i = (int32_t*)(b + w.ring_i);
    ring_rows = w.ring_rows;
    sub_vn = (double*)(b + w.sub_vn);
    sub_vd = (double*)(b + w.sub_vd);
    sub_vl = (int32_t*)(b + w.sub_vl);
    sub_vi = (int32_t*)(b + w.sub_vi);
    sub_mab = (int32_t*)(b + w.sub_mab);
    sub_md = (double*)(b + w.sub_md);
    sub_don = (int32_t*)(b + w.sub_don);
    sub_dd = (double*)(b + w.sub_dd);
    sub_gab = (int32_t*)(b + w.sub_gab);
    sub_gd = (double*)(b + w.sub_gd);
    sub_gdon = (int32_t*)(b + w.sub_gdon);
    sub_gdd = (double*)(b + w.sub_gdd);
    delta = fp32 ? (float*)(b + w.delta) : nullptr;
    hard = fp32 ? (int32_t*)(b + w.hard) : nullptr;
    if (P->cfg.mset_radius > 0.0) {
      ms.meta = (double*)(b + w.ms_meta);
      ms.count = (uint32_t*)(b + w.ms_count);
      ms.keys0 = (uint64_t*)(b + w.ms_keys0);
      ms.keys1 = (uint64_t*)(b + w.ms_keys1);
      ms.vals0 = (double*)(b + w.ms_vals0);
      ms.vals1 = (double*)(b + w.ms_vals1);
      ms.hist = (uint32_t*)(b + w.ms_hist);
      ms.taken = (uint64_t*)(b + w.ms_taken);
      ms.bucket = (uint32_t*)(b + w.ms_bucket);
    }
  }

  bool chk(hipError_t e) {
    if (err == hipSuccess && e != hipSuccess) err = e;
    return err == hipSuccess;
  }

  Status advance();
};

#define LCHECK(expr)                 \
  do {                               \
    if (!chk(expr)) return DONE;     \
  } while (0)

LaneRun::Status LaneRun::advance() {
  if (err != hipSuccess || si >= ln->series.size()) return DONE;
  hipStream_t st = run_st;
  const int s = ln->series[si];
  const valmod_layout& Ls = P->lay[s];
  const PassGeom& G = P->geom[s];
  const int64_t n = Ls.n, N0 = Ls.n0;
  const int esz = P->cfg.dtype == VALMOD_F32 ? 4 : 8;
  const int excl_den = P->cfg.excl_den;
  const bool fp32 = P->cfg.precision == VALMOD_PREC_FP32_REFRESH;
  // the series' outputs; those the caller skips (null) but the run reads back
  // live in the workspace
  double* vnorm = o->valmp_norm ? o->valmp_norm + Ls.valmp : sub_vn;
  double* vdist = o->valmp_dist ? o->valmp_dist + Ls.valmp : sub_vd;
  int32_t* vlen = o->valmp_len ? o->valmp_len + Ls.valmp : sub_vl;
  int32_t* vidx = o->valmp_idx ? o->valmp_idx + Ls.valmp : sub_vi;
  int32_t* mot_ab = o->motif_ab ? o->motif_ab + 2 * Ls.motif : sub_mab;
  double* mot_d = o->motif_d ? o->motif_d + Ls.motif : sub_md;
  int32_t* dis_on = o->discord_on ? o->discord_on + 2 * Ls.discord : sub_don;
  double* dis_d = o->discord_d ? o->discord_d + Ls.discord : sub_dd;
  int32_t* g_mab = o->g_motif_abl ? o->g_motif_abl + 3 * Ls.g_motif : sub_gab;
  double* g_md = o->g_motif_d ? o->g_motif_d + 2 * Ls.g_motif : sub_gd;
  int32_t* g_don = o->g_discord_onl ? o->g_discord_onl + 3 * Ls.g_discord : sub_gdon;
  double* g_dd = o->g_discord_d ? o->g_discord_d + 2 * Ls.g_discord : sub_gdd;
  if (!open) {
    const char* series = d_series + (size_t)Ls.series * esz;
    LCHECK(launch_convert(series, P->cfg.dtype, n, n + kPad, xs, (int*)&cnt[CNT_ERR], st));
    LCHECK(launch_valmp_init(N0, vnorm, vdist, vlen, vidx, st));
    // partial profiles are used unless every length is forced through a full pass
    heaps_on = P->cfg.path != VALMOD_PATH_FULL && Ls.l_max > Ls.l_min && !noalloc && !P->tune_no_heaps;
    base = 0;            // base length of the current partial profiles (0: none)
    probe_next = false;  // judge the partial profiles at the first length after a rebuild
    L = Ls.l_min;
    anc_len = 0;
    phase = 0;
    open = true;
  }
  // FP32 work items whose rounding bound exceeds this go to the FP64 kernel
  const float delta_max = (float)(env_int("VALMOD_FP32_DELTA_MAX_E6", 5000) * 1.0e-6);
  const int p = P->cfg.p;
  const int D = p < 15 ? p : 15;
  // rounding bound of a correlation evaluated directly from anchored sums
  const double margin = direct_bound(L);
  const double rec_factor = env_int("VALMOD_RECOMPUTE_FACTOR_X100", 80) / 100.0;
  const int64_t t = L - Ls.l_min;
  const int64_t N = n - L + 1;
  const int64_t e = excl_zone(L, excl_den);
  const PassGrid grid = pass_grid(N, e, G.dstart, G.K, G.H);
  // dense dot-product blocks (anchor table, row recompute) on FP64 matrix cores;
  // VALMOD_MFMA=0 selects the VALU kernels
  const bool use_mfma = env_int("VALMOD_MFMA", 1) != 0;
  // exact rows of the listed owners (every eligible candidate), reduced into `best`
  auto recompute_rows = [&](const int32_t* list, const unsigned long long* nlist) -> hipError_t {
    return use_mfma ? launch_recompute_mfma(xs, A, invn, flat, list, nlist, N, N, L, e, best, st)
                    : launch_recompute(xs, A, invn, flat, list, nlist, N, N, L, e, best, st);
  };
  // m-th discords from the partial profiles: each owner's m best stored
  // candidates and whether the bound of the unstored ones certifies them
  const int md = P->cfg.m_discords;
  auto mth_select = [&](bool fresh) -> hipError_t {
    MthSelect ms_{};
    ms_.A = A;
    ms_.invn = invn;
    ms_.sig = sig;
    ms_.flat = flat;
    ms_.hc = hc;
    ms_.hn = hn;
    ms_.hS = hS;
    ms_.hbound = hbound;
    ms_.hsig = hsig;
    ms_.rflat = &cnt[CNT_RFLAT];
    ms_.fresh = fresh ? 1 : 0;
    ms_.p = p;
    ms_.m = md;
    ms_.N = N;
    ms_.N0 = N0;
    ms_.L = L;
    ms_.e = e;
    ms_.base = base;
    ms_.margin = margin;
    ms_.vals = mvals;
    ms_.nn = mnn;
    ms_.ub = mub;
    ms_.mstate = mstate;
    ms_.n_open = &cnt[CNT_MOPEN];
    return launch_mth_select(ms_, st);
  };
  // this length's profile row in the ring (and in the outputs unless skipped)
  double* rd = ring_d + (t % ring_rows) * N0;
  int32_t* ri = ring_i + (t % ring_rows) * N0;
  double* pd = o->prof_dist ? o->prof_dist + Ls.prof + t * N0 : nullptr;
  int32_t* pi = o->prof_idx ? o->prof_idx + Ls.prof + t * N0 : nullptr;
  const int32_t* prev = L > Ls.l_min ? ring_i + ((t - 1) % ring_rows) * N0 : nullptr;

  const bool sweep = heaps_on && base > 0 && L > Ls.l_min;
  if (phase == 0) {
    // statistics, recurrence inputs and FP32 copies at L; the sums of L go to the
    // other buffer, which then becomes the current one
    WindowPrep wpr{};
    wpr.xs = xs;
    wpr.N = N;
    wpr.L = L;
    wpr.first = L == Ls.l_min ? 1 : 0;
    wpr.flat_eps = P->cfg.flat_eps;
    wpr.A_in = A;
    wpr.B_in = B;
    wpr.A_out = A2;
    wpr.B_out = B2;
    wpr.mu = mu;
    wpr.sig = sig;
    wpr.invn = invn;
    wpr.flat = flat;
    wpr.nflat = &cnt[CNT_NFLAT];
    wpr.df = df;
    wpr.dg = dg;
    wpr.sw32 = sw32;
    if (fp32) {
      wpr.df32 = df32;
      wpr.dg32 = dg32;
      wpr.inv32 = inv32;
    }
    wpr.bsw_max = bsw_max;
    wpr.bsw_min = bsw_min;
    wpr.bdf_max = bdf_max;
    wpr.bdg_max = bdg_max;
    wpr.bmu_max = bmu_max;
    if (sweep) {  // windows flat at the base length that are candidates at L
      wpr.hflat = hflat;
      wpr.hsig = hsig;
      wpr.rflat = &cnt[CNT_RFLAT];
    }
    LCHECK(launch_window_prep(wpr, st));
    std::swap(A, A2);
    std::swap(B, B2);
    // the anchor table at L: formed at the first length, else moved on by one
    // term unless the last pass of the previous length did so
    if (G.table && anc_len != L) {
      // first length: the Hankel-block contraction on FP64 matrix cores; later
      // lengths add one term per anchor
      if (L == Ls.l_min && use_mfma)
        LCHECK(launch_anchor_mfma(xs, n, L, G.H, G.dstart, G.segs, G.stride, G.stride, anc, st));
      else
        LCHECK(launch_anchor(xs, n, L, L == Ls.l_min, G.H, G.dstart, G.segs, G.stride, G.stride, anc, st));
      anc_len = L;
    }
    if (sweep) {
      // Alg. ComputeSubMP: sweep the partial profiles, certify by the lower bound;
      // the choice between row recompute and a full pass needs the counts
      if (lbm) LCHECK(launch_fill_counters(&cnt[CNT_MINDIST], 2, 0x7FF0000000000000ull, st));  // +inf
      LCHECK(launch_sweep(xs, A, invn, sig, flat, N, L, e, p, base, hc, hS, hn, hbound, hsig, &cnt[CNT_RFLAT], margin,
                          best, fail,
                          &cnt[CNT_NFAIL], &cnt[CNT_VALID], lbm, lbm ? &cnt[CNT_MINDIST] : nullptr,
                          lbm ? &cnt[CNT_MINLB] : nullptr, st));
      if (capture) {
        err = hipErrorNotSupported;  // unreachable: a captured plan has no partial profiles
        return DONE;
      }
      if (md > 1) {
        LCHECK(launch_zero_counters(&cnt[CNT_MOPEN], 1, st));
        LCHECK(mth_select(false));
      }
      // NFAIL, VALID, HARD, BIG, MINDIST, MINLB (and MOPEN)
      LCHECK(hipMemcpyAsync(ln->hcnt, &cnt[CNT_NFAIL], 6 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
      if (md > 1) LCHECK(hipMemcpyAsync(ln->hcnt + 6, &cnt[CNT_MOPEN], sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
      LCHECK(hipMemcpyAsync(ln->hcnt + kOverSlot, &cnt[CNT_OVER], sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            st));
      LCHECK(hipEventRecord(ln->ready, st));
      phase = 1;
      return BLOCKED;
    }
  }

  PassLaunch pl{};
  pl.xs = xs;
  pl.mu = mu;
  pl.df = df;
  pl.dg = dg;
  pl.sw32 = sw32;
  pl.invn = invn;
  pl.df32 = df32;
  pl.dg32 = dg32;
  pl.inv32 = inv32;
  pl.thr = thr;
  pl.thr32 = thr32;
  pl.best = best;
  pl.anc = G.table ? anc : nullptr;
  pl.A = A;
  pl.anc_stride = G.stride;
  pl.N = N;
  pl.e = e;
  pl.H = G.H;
  pl.dstart = G.dstart;
  pl.L = L;
  pl.K = G.K;
  pl.events = &cnt[CNT_EV_STEPS];
  pl.cnt = acnt;
  pl.buf = abuf;
  pl.cap = P->cap;
  int64_t passes = 0;
  // full-grid launch of the plan's own pass kernel, timed by events that the
  // launch records itself (kernel start and end)
  auto timed_pass = [&](const PassLaunch& q) -> hipError_t {
    const bool tm = !capture && !noalloc && evi + 2 <= (int64_t)ln->ev.size();
    PassLaunch qt = q;
    if (tm) {
      qt.ev_start = ln->ev[evi];
      qt.ev_stop = ln->ev[evi + 1];
      evi += 2;
    }
    const hipError_t e1 = launch_pass(qt, st);
    P->pass_launches += 1;
    P->pass_cells += grid.cells;
    ++passes;
    return e1;
  };
  bool bounds_ready = false;
  // per-item rounding bounds of the recurrence at this length (their inputs come
  // from the window prep): FP64 always; FP32 items over the limit are listed for
  // the FP64 kernel
  auto bounds_setup = [&]() -> hipError_t {
    if (bounds_ready) return hipSuccess;
    bounds_ready = true;
    return launch_item_bounds(bsw_max, bsw_min, bdf_max, bdg_max, bmu_max, N, e, G.dstart, G.K, G.H, L, delta_max,
                              delta64,
                              fp32 ? delta : nullptr, hard, &cnt[CNT_HARD], st);
  };
  bool recompute = false;  // process the recompute list (its length is a device counter)
  bool grow_collect = false;  // the collecting pass is the length's last and moves the anchor table on
  // collecting pass above per-owner thresholds from the candidates of `src`,
  // then the exact merge (top-`keep` partial profiles and best keys)
  bool fail_reset = sweep;  // the sweep's recompute list, replaced by the first collecting pass
  bool tighten = false;     // the collecting pass with p thresholds takes the replaced profiles' thresholds too
  bool count_over = false;  // that pass counts the owners whose list overflows (CNT_OVER)
  auto collect = [&](const int32_t* src, int p_eff, int keep, int best_exact) -> hipError_t {
    // the wavefront-per-owner merge list is rebuilt by every collecting pass (a
    // length may run two); the recompute list keeps the owners listed so far at
    // this length, except the sweep's, which the first collecting pass replaces
    hipError_t e1 = launch_zero_counters(&cnt[CNT_BIG], 1, st);
    if (e1 == hipSuccess && fail_reset) e1 = launch_zero_counters(&cnt[CNT_NFAIL], 1, st);
    fail_reset = false;
    if (e1 == hipSuccess)
      e1 = launch_seed_append(xs, A, invn, flat, src, N, L, e, p_eff, p_eff == 1 ? 0 : D, margin, best_exact, thr,
                              fp32 ? thr32 : nullptr, acnt, fail, &cnt[CNT_NFAIL], st);
    if (e1 == hipSuccess && tighten && p_eff == p)
      e1 = launch_tighten_threshold(thrp, N, thr, fp32 ? thr32 : nullptr, st);
    PassLaunch q = pl;
    q.append = true;
    q.grow = grow_collect;
    if (e1 == hipSuccess) e1 = bounds_setup();
    if (fp32) {
      q.fp32 = true;
      q.delta = delta;
      q.delta_max = delta_max;
      if (e1 == hipSuccess) e1 = timed_pass(q);
      // then the listed items in FP64 (a small grid that walks the device-side
      // list; on the same stream: a second stream's fork and join cost more
      // than the overlap gained, since the list is usually empty)
      PassLaunch h = pl;
      h.append = true;
      h.items = hard;
      h.nitems = grid.segs * grid.bands;
      h.nitems_dev = &cnt[CNT_HARD];
      h.grow = grow_collect;  // the items the FP32 pass left (disjoint anchors)
      h.delta = delta64;
      h.delta_max = INFINITY;
      if (e1 == hipSuccess) e1 = launch_pass(h, st);
      ++passes;
    } else if (e1 == hipSuccess) {
      q.delta = delta64;
      q.delta_max = INFINITY;
      e1 = timed_pass(q);
    }
    if (e1 == hipSuccess)
      e1 = launch_merge(xs, A, invn, sig, flat, thr, acnt, abuf, P->cap, N, L, p, keep, margin, best_exact, hc, hS,
                        hn, hbound, hsig, hflat, best, fail, &cnt[CNT_NFAIL], big, &cnt[CNT_BIG], &cnt[CNT_APPENDS],
                        count_over && p_eff == p ? &cnt[CNT_OVER] : nullptr, st);
    recompute = true;
    return e1;
  };

  int64_t nvalid = 0, nswept_fail = 0;
  bool full = true, rebuild = false;
  int mth = 0;  // m-th discords from the partial profiles: 1 after a sweep, 2 after a rebuild
  int paper_split = 0;  // paper mode: 1 recompute the failing owners below minDistAbs, 2 leave all partial
  if (L == Ls.l_min) {
    rebuild = heaps_on;
  } else if (sweep && P->cfg.mode == VALMOD_MODE_PAPER) {
    // Alg. ComputeSubMP: the motif is certified when the best certified distance is below
    // every failing owner's bound; otherwise, when the failing owners are few
    // (fewer than N log p / log N), only those whose bound is below it are recomputed;
    // otherwise a full pass rebuilds the partial profiles at L (Alg. VALMOD)
    nswept_fail = (int64_t)ln->hcnt[0];
    nvalid = (int64_t)ln->hcnt[1];
    uint64_t bd = ln->hcnt[4], bl = ln->hcnt[5];
    double min_dist_abs, min_lb_abs;
    memcpy(&min_dist_abs, &bd, 8);
    memcpy(&min_lb_abs, &bl, 8);
    const double limit = (double)N * log((double)(p > 1 ? p : 2)) / log((double)(N > 2 ? N : 3));
    // the published limit weighs an O(n log n) profile against the matrix profile;
    // here a recomputed row costs N L multiply-adds against N^2 / 2 cells of a
    // full pass, so a full pass is also taken when the rows would cost more
    const double cells = 0.5 * (double)N * (double)N;
    const bool rows_cheap = (double)nswept_fail * (double)N * (double)L <= rec_factor * cells;
    if (min_dist_abs < min_lb_abs) {
      full = false;
      paper_split = 2;
    } else if ((double)nswept_fail < limit && rows_cheap) {
      full = false;
      paper_split = 1;
    } else {
      rebuild = true;
    }
  } else if (sweep) {
    nswept_fail = (int64_t)ln->hcnt[0];
    nvalid = (int64_t)ln->hcnt[1];
    // row recompute of the failing windows vs one full pass (cost model in
    // FMA-equivalents); with m-th discords at most m rows for every owner whose
    // m-list is not certified
    const double cells = 0.5 * (double)N * (double)N;
    const double rows = md > 1 ? (double)md * (double)ln->hcnt[6] : (double)nswept_fail;
    const bool cheap = rows * (double)N * (double)L <= rec_factor * cells;
    if (P->cfg.path == VALMOD_PATH_RECOMPUTE || cheap) {
      full = false;
      recompute = nswept_fail > 0;
      if (md > 1) mth = 1;
    } else if (probe_next && (double)nswept_fail > 0.25 * (double)N) {
      heaps_on = false;  // the bound fails right after a rebuild: partial profiles do not pay here
    } else {
      rebuild = true;
    }
    probe_next = false;
  }
  if (full) {
    const int32_t* src = prev;
    // Every length's neighbours come from a collecting pass: the recurrence (in
    // either precision) only selects the candidates that its rounding bound
    // cannot exclude, and the merge evaluates them directly. At the first length
    // an FP64 matrix-profile pass (running best keys) provides the seeds. The
    // collecting pass is the length's last and moves the anchor table on to L + 1.
    const bool grow = G.table && anc_len == L && L < Ls.l_max;
    grow_collect = grow;
    if (L == Ls.l_min) {
      LCHECK(launch_seed_mp(xs, mu, invn, flat, nullptr, N, L, e, best, thr, thr32, st));
      PassLaunch q = pl;
      q.append = false;
      q.grow = false;
      LCHECK(launch_pass(q, st));
      ++passes;
      LCHECK(launch_keys_to_idx(best, N, ri, st));
      src = ri;
    }
    if (rebuild) {
      // thresholds from the partial profiles being replaced (the sweep grew their
      // sums to L; an overflowed list left the best p of its first candidates),
      // taken before a collecting pass overwrites the profiles. Once a rebuild has
      // run with them, few lists of the pass with p thresholds overflow: that pass
      // alone then gives the exact neighbours (the owners whose list overflows go
      // to the row recompute) when the previous rebuild's overflowing lists would
      // cost less to recompute than a full pass
      bool one = false;
      if (sweep) {
        LCHECK(launch_profile_threshold(A, invn, flat, hc, hS, hn, p, N, L, e, margin, thrp, st));
        tighten = true;
        const double over_rows = (double)ln->hcnt[kOverSlot];
        one = md == 1 && over_rows * (double)N * (double)L <= rec_factor * 0.5 * (double)N * (double)N;
      }
      LCHECK(launch_zero_counters(&cnt[CNT_OVER], 1, st));
      count_over = true;
      if (!one) {
        // exact neighbours first (a list of one threshold rarely overflows), so
        // that the owners whose partial-profile list overflows keep them: on
        // periodic series the p-th best seed is far below the p-th best
        // candidate, and without the replaced profiles' thresholds the lists of
        // nearly all owners overflow
        grow_collect = false;
        LCHECK(collect(src, 1, 0, 0));
        LCHECK(launch_keys_to_idx(best, N, ri, st));
        src = ri;
      }
      grow_collect = grow;
      // new partial profiles at base L (Alg. ComputeMatrixProfile); with two
      // passes `best` already holds the exact neighbours
      LCHECK(collect(src, p, p, one ? 0 : 1));
      base = L;
      probe_next = true;
      if (md > 1) mth = 2;
    } else if (md > 1) {
      // exact top-m lists of every owner (Def. m-th best match)
      LCHECK(collect(src, md, md, 0));
    } else {
      // exact neighbours, seeded by the previous length (or the first length's pass)
      LCHECK(collect(src, 1, 0, 0));
    }
    if (grow) anc_len = L + 1;
  }
  if (paper_split) {
    LCHECK(launch_split_fail(fail, &cnt[CNT_NFAIL], N, lbm, &cnt[CNT_MINDIST], paper_split == 2 ? 1 : 0, rec,
                             &cnt[CNT_NREC], part, &cnt[CNT_NPART], st));
    if (paper_split == 1) LCHECK(recompute_rows(rec, &cnt[CNT_NREC]));
  }
  if (mth) {
    // Alg. Topkm_nextLength: owners whose m-list the partial profiles certify
    // enter the rankings as they are; the cutoff from their rankings (twice the
    // exclusion zone) leaves out the uncertified owners that cannot reach the
    // top k of any column, and the rest get a top-m row recompute. After a
    // sweep, the best-match recompute list becomes the pruned owners whose best
    // match the sweep did not certify.
    const int kd = P->cfg.k_discords;
    const bool fresh = mth == 2;
    if (fresh) LCHECK(mth_select(true));
    LCHECK(launch_mth_rankings(mvals, mnn, N0, n, L, md, excl_den, kd, tau_on, tau_d, st, 2));
    if (!fresh) LCHECK(launch_zero_counters(&cnt[CNT_NFAIL], 1, st));
    LCHECK(launch_mth_prune(mstate, mub, tau_d, N, N0, md, kd, fresh ? 1 : 0, mlist, &cnt[CNT_MREC], fail,
                            &cnt[CNT_NFAIL], &cnt[CNT_MCERT], &cnt[CNT_MPRUNED], st));
    LCHECK(launch_recompute_topm_keys(xs, A, invn, flat, mlist, &cnt[CNT_MREC], N, N, N0, L, e, md, mkeys, best,
                                      mvals, mnn, use_mfma, st));
    if (!fresh) recompute = true;
    if (recompute) LCHECK(recompute_rows(fail, &cnt[CNT_NFAIL]));
  } else if (recompute && md > 1) {
    LCHECK(launch_recompute_topm(xs, A, invn, flat, fail, &cnt[CNT_NFAIL], N, N, L, e, md, p, mkeys, hc, hS, hn, best,
                                 use_mfma, st));
  } else if (recompute) {
    LCHECK(recompute_rows(fail, &cnt[CNT_NFAIL]));
  }
  LCHECK(launch_finalize(xs, mu, sig, best, N, N0, L, rd, ri, pd, pi, vnorm, vdist, vlen, vidx, st));
  if (md > 1) {
    const int kd = P->cfg.k_discords;
    const int64_t at = Ls.mdiscord + t * md * kd;
    if (!mth) LCHECK(launch_mth_values(A, invn, flat, hc, hS, hn, p, md, N, N0, L, mvals, mnn, st));
    LCHECK(launch_mth_rankings(mvals, mnn, N0, n, L, md, excl_den, kd, o->mdiscord_on + 2 * at, o->mdiscord_d + at,
                               st));
  }
  if (paper_split) {
    LCHECK(launch_mark_partial(part, &cnt[CNT_NPART], N, lbm, rd, ri, st));
    if (pd || pi) LCHECK(launch_mark_partial(part, &cnt[CNT_NPART], N, lbm, pd, pi, st));
  }
  // per-length rankings of the ring's rows, a group of lengths at a time (one
  // workgroup per length)
  if (t % ring_rows == ring_rows - 1 || L == Ls.l_max) {
    const int64_t t0 = t - t % ring_rows;
    const int km = P->cfg.k_motifs, kd = P->cfg.k_discords;
    LCHECK(launch_rankings(ring_d, ring_i, N0, n, (int)(Ls.l_min + t0), (int)(t - t0 + 1), excl_den, km, kd,
                           mot_ab + 2 * t0 * km, mot_d + t0 * km, dis_on + 2 * t0 * kd, dis_d + t0 * kd, st));
  }
  LCHECK(launch_record_stats(cnt, o->stats ? o->stats + Ls.stats + t * VALMOD_NSTATS : nullptr, full ? 1 : 0,
                             nvalid, nswept_fail, paper_split == 1 ? 2 : (recompute ? 1 : 0), passes,
                             rebuild ? 1 : 0, st));
  // VALMOD_PROGRESS=k: one line on stderr every k lengths, once the length has run
  const int progress = capture || noalloc ? 0 : env_int("VALMOD_PROGRESS", 0);
  if (progress > 0 && (t % progress == 0 || L == Ls.l_max)) {
    LCHECK(hipStreamSynchronize(st));
    fprintf(stderr, "valmod: series %d length %d (%lld of %lld) done, heaps %s\n", s, L, (long long)t + 1,
            (long long)Ls.nlen, heaps_on ? "on" : "off");
    fflush(stderr);
  }
  phase = 0;
  if (++L > Ls.l_max) {
    const int km = P->cfg.k_motifs, kd = P->cfg.k_discords;
    LCHECK(launch_global_rank(vnorm, vdist, vlen, vidx, N0, dis_on, dis_d, (int)Ls.nlen, Ls.l_min, excl_den, km, kd,
                              g_mab, g_md, g_don, g_dd, st));
    if (P->cfg.mset_radius > 0.0) {
      // motif sets of the global top-k pairs (Sec. "Finding Motif Sets")
      ms.xs = xs;
      ms.n = n;
      ms.n0 = N0;
      ms.abl = g_mab;
      ms.gd = g_md;
      ms.k = km;
      ms.D = P->cfg.mset_radius;
      ms.excl_den = excl_den;
      ms.flat_eps = P->cfg.flat_eps;
      ms.cap = P->cfg.mset_cap;
      ms.cand_cap = (int64_t)km * N0;
      ms.out_count = o->mset_count + Ls.g_motif;
      ms.out_off = o->mset_off + Ls.mset;
      ms.out_dist = o->mset_dist + Ls.mset;
      LCHECK(launch_motif_sets(ms, st));
    }
    if (md > 1)
      LCHECK(launch_mth_global(o->mdiscord_on + 2 * Ls.mdiscord, o->mdiscord_d + Ls.mdiscord, (int)Ls.nlen, Ls.l_min,
                               md, kd, o->g_mdiscord_onl + 3 * Ls.g_mdiscord, o->g_mdiscord_d + 2 * Ls.g_mdiscord,
                               st));
    open = false;
    ++si;
  }
  return CONTINUE;
}

#undef LCHECK

// Enqueues the whole run: the lanes fork from the caller's stream, advance one
// length at a time in turn (a blocked lane is skipped until its counters have
// arrived), and join back into the caller's stream.
hipError_t enqueue_run(valmod_plan_s* P, char* ws, const valmod_outputs* o, const char* d_series, hipStream_t st,
                       bool capture) {
  hipError_t e = hipEventRecord(P->start, st);
  std::vector<LaneRun> runs(P->lanes.size());
  for (size_t l = 0; e == hipSuccess && l < P->lanes.size(); ++l) {
    Lane& ln = P->lanes[l];
    runs[l].init(P, &ln, ws, o, d_series, capture);
    e = hipStreamWaitEvent(ln.st, P->start, 0);
    if (e == hipSuccess)
      e = launch_zero_counters((unsigned long long*)(ws + ln.base + ln.ws.counters), CNT_WORDS, ln.st);
  }
  std::vector<char> done(P->lanes.size(), 0), blocked(P->lanes.size(), 0);
  size_t remaining = e == hipSuccess ? P->lanes.size() : 0;
  while (remaining > 0) {
    bool progressed = false;
    int first_blocked = -1;
    for (size_t l = 0; l < P->lanes.size(); ++l) {
      if (done[l]) continue;
      if (blocked[l]) {
        const hipError_t q = hipEventQuery(P->lanes[l].ready);
        if (q == hipErrorNotReady) {
          if (first_blocked < 0) first_blocked = (int)l;
          continue;
        }
        if (q != hipSuccess) {
          e = q;
          remaining = 0;
          break;
        }
        blocked[l] = 0;
      }
      const LaneRun::Status r = runs[l].advance();
      progressed = true;
      if (r == LaneRun::DONE) {
        done[l] = 1;
        --remaining;
      } else if (r == LaneRun::BLOCKED) {
        blocked[l] = 1;
      }
    }
    if (!progressed && first_blocked >= 0) {
      e = hipEventSynchronize(P->lanes[first_blocked].ready);
      if (e != hipSuccess) break;
    }
  }
  for (size_t l = 0; l < runs.size(); ++l) {
    if (e == hipSuccess && runs[l].err != hipSuccess) e = runs[l].err;
    P->lanes[l].nev = runs[l].evi;
  }
  for (size_t l = 0; l < P->lanes.size(); ++l) {
    Lane& ln = P->lanes[l];
    if (e == hipSuccess) e = hipEventRecord(ln.done, ln.st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ln.done, 0);
  }
  return e;
}

}  // namespace

extern "C" valmod_status valmod_run(valmod_plan_t P, const void* d_series, void* d_ws,
                                    const valmod_outputs* o, void* stream_) {
  if (!P || !d_series || !d_ws || !o) return VALMOD_E_ARG;
  if (((uintptr_t)d_ws) % kAlign) return VALMOD_E_ARG;
  if (P->cfg.m_discords > 1 && (!o->mdiscord_on || !o->mdiscord_d || !o->g_mdiscord_onl || !o->g_mdiscord_d))
    return VALMOD_E_ARG;
  if (P->cfg.mset_radius > 0.0 && (!o->mset_count || !o->mset_off || !o->mset_dist)) return VALMOD_E_ARG;
  hipStream_t st = (hipStream_t)stream_;
  int prev_dev = -1;
  if (hipGetDevice(&prev_dev) != hipSuccess) return VALMOD_E_HIP;
  if (hipSetDevice(P->cfg.device) != hipSuccess) return VALMOD_E_HIP;
  char* ws = (char*)d_ws;
  hipError_t e = ensure_resources(P);
  P->pass_ms = 0.0;
  P->pass_launches = 0;
  P->pass_cells = 0;
  P->run_pending = false;
  P->na_pending = false;
  if (e == hipSuccess && P->cfg.graph) {
    // one captured graph per set of buffers and stream, replayed on later calls
    const bool same = P->exec && P->key_series == d_series && P->key_ws == d_ws && P->key_stream == st &&
                      memcmp(&P->key_out, o, sizeof(*o)) == 0;
    if (!same) {
      if (P->exec) (void)hipGraphExecDestroy(P->exec);
      P->exec = nullptr;
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        const hipError_t e1 = enqueue_run(P, ws, o, (const char*)d_series, st, true);
        e = hipStreamEndCapture(st, &g);
        if (e1 != hipSuccess) e = e1;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e == hipSuccess) {
        P->key_series = d_series;
        P->key_ws = d_ws;
        P->key_stream = st;
        P->key_out = *o;
        P->graph_cells = P->pass_cells;
      }
    }
    if (e == hipSuccess) e = hipEventRecord(P->g0, st);
    if (e == hipSuccess) e = hipGraphLaunch(P->exec, st);
    if (e == hipSuccess) e = hipEventRecord(P->g1, st);
  } else if (e == hipSuccess) {
    e = enqueue_run(P, ws, o, (const char*)d_series, st, false);
  }
  // device error flags of every lane, read by valmod_run_status
  for (Lane& ln : P->lanes)
    if (e == hipSuccess)
      e = hipMemcpyAsync(&ln.hcnt[kErrSlot], ws + ln.base + ln.ws.counters + CNT_ERR * 8, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(P->finished, st);
  if (e == hipSuccess) P->run_pending = true;
  (void)hipSetDevice(prev_dev);
  return e == hipSuccess ? VALMOD_OK : VALMOD_E_HIP;
}

extern "C" valmod_status valmod_run_status(valmod_plan_t P, void* stream_) {
  if (!P) return VALMOD_E_ARG;
  if (P->na_pending) {
    // a run of valmod_run_noalloc: its error flags sit in the static scratch
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return VALMOD_E_HIP;
    if (hipSetDevice(P->cfg.device) != hipSuccess) return VALMOD_E_HIP;
    hipError_t e = hipStreamSynchronize(stream_ ? (hipStream_t)stream_ : P->na_stream);
    valmod_status status = VALMOD_OK;
    for (Lane& ln : P->lanes) {
      unsigned long long flag = 0;
      if (e == hipSuccess)
        e = hipMemcpy(&flag, P->na_ws + ln.base + ln.ws.counters + CNT_ERR * 8, 8, hipMemcpyDeviceToHost);
      if (e == hipSuccess && flag) status = VALMOD_E_DEVICE;
    }
    if (e != hipSuccess) status = VALMOD_E_HIP;
    P->pass_ms = 0.0;  // no timing events in this mode
    P->na_pending = false;
    P->last_status = status;
    (void)hipSetDevice(prev);
    return status;
  }
  if (!P->run_pending) return P->last_status;
  int prev_dev = -1;
  if (hipGetDevice(&prev_dev) != hipSuccess) return VALMOD_E_HIP;
  if (hipSetDevice(P->cfg.device) != hipSuccess) return VALMOD_E_HIP;
  hipError_t e = stream_ ? hipStreamSynchronize((hipStream_t)stream_) : hipSuccess;
  if (e == hipSuccess) e = hipEventSynchronize(P->finished);
  P->pass_ms = 0.0;
  if (e == hipSuccess && P->cfg.graph) {
    // graph mode reports the whole replay as one launch
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, P->g0, P->g1);
    P->pass_ms = ms;
    P->pass_launches = 1;
    P->pass_cells = P->graph_cells;
  } else if (e == hipSuccess) {
    for (Lane& ln : P->lanes)
      for (int64_t i = 0; e == hipSuccess && i + 1 < ln.nev; i += 2) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ln.ev[i], ln.ev[i + 1]);
        P->pass_ms += ms;
      }
  }
  valmod_status status = VALMOD_OK;
  if (e != hipSuccess) {
    status = VALMOD_E_HIP;
  } else {
    for (Lane& ln : P->lanes)
      if (ln.hcnt[kErrSlot]) status = VALMOD_E_DEVICE;
  }
  P->run_pending = false;
  P->last_status = status;
  (void)hipSetDevice(prev_dev);
  return status;
}

// The run of valmod_run on the static scratch: every lane in turn on the
// caller's stream, full diagonal pass at every length (no host decisions), no
// lane streams, events or pinned memory, and no allocation of any kind.
extern "C" valmod_status valmod_run_noalloc(valmod_plan_t P, const void* d_series, const valmod_outputs* o,
                                            void* stream_) {
  if (!P || !d_series || !o) return VALMOD_E_ARG;
  if (P->ws_total > (size_t)VALMOD_NOALLOC_SCRATCH_BYTES) return VALMOD_E_SCRATCH;
  if (P->cfg.mode == VALMOD_MODE_PAPER) return VALMOD_E_ARG;  // needs host decisions
  if (P->cfg.m_discords > 1 && (!o->mdiscord_on || !o->mdiscord_d || !o->g_mdiscord_onl || !o->g_mdiscord_d))
    return VALMOD_E_ARG;
  if (P->cfg.mset_radius > 0.0 && (!o->mset_count || !o->mset_off || !o->mset_dist)) return VALMOD_E_ARG;
  hipStream_t st = (hipStream_t)stream_;
  int prev_dev = -1;
  if (hipGetDevice(&prev_dev) != hipSuccess) return VALMOD_E_HIP;
  if (hipSetDevice(P->cfg.device) != hipSuccess) return VALMOD_E_HIP;
  void* ws = nullptr;
  hipError_t e = scratch_address(P->cfg.device, &ws);
  P->pass_ms = 0.0;
  P->pass_launches = 0;
  P->pass_cells = 0;
  P->run_pending = false;
  P->na_pending = false;
  for (Lane& ln : P->lanes) {
    if (e != hipSuccess) break;
    LaneRun r;
    r.init(P, &ln, (char*)ws, o, (const char*)d_series, false);
    r.noalloc = true;
    r.run_st = st;
    e = launch_zero_counters((unsigned long long*)((char*)ws + ln.base + ln.ws.counters), CNT_WORDS, st);
    // no partial profiles, so no length waits for device counters: a lane only
    // continues or finishes
    while (e == hipSuccess) {
      const LaneRun::Status rs = r.advance();
      if (rs == LaneRun::DONE) break;
      if (rs == LaneRun::BLOCKED) e = hipErrorNotSupported;
    }
    if (e == hipSuccess) e = r.err;
  }
  if (e == hipSuccess) {
    P->na_pending = true;
    P->na_ws = (char*)ws;
    P->na_stream = st;
  }
  (void)hipSetDevice(prev_dev);
  return e == hipSuccess ? VALMOD_OK : VALMOD_E_HIP;
}

// Empirical choice of the pass geometry and of p on the series with the most
// work. Stage 1 (geometry: FP64 segment height, FP32 refresh interval, and
// diagonals per lane) times each candidate on two slices of three lengths, at
// the start and at the end of the length range, on the full path. Stage 2
// (exact mode with partial profiles only) times p, p/2 and p/4 on the first four
// lengths with the plan's own path: the outputs do not depend on p there, but the
// cost of building the partial profiles and what they save do. Each measurement
// is the second of two runs; the fastest candidate whose workspace fits is kept.
// The tuning runs write no output.
extern "C" valmod_status valmod_autotune(valmod_plan_t P, const void* d_series, void* d_ws, const valmod_outputs* o,
                                         void* stream, int32_t* chosen) {
  (void)o;  // the tuning runs skip every output
  if (!P || !d_series || !d_ws) return VALMOD_E_ARG;
  const bool fp32 = P->cfg.precision == VALMOD_PREC_FP32_REFRESH;
  int sbest = 0;
  double cbest = -1.0;
  for (int s = 0; s < P->cfg.num_series; ++s) {
    double c = 0.0;
    for (int64_t L = P->lmin[s]; L <= P->lmax[s]; ++L) c += (double)(P->n[s] - L + 1) * (double)(P->n[s] - L + 1);
    if (c > cbest) {
      cbest = c;
      sbest = s;
    }
  }
  const valmod_layout& Ls = P->lay[sbest];
  const int esz = P->cfg.dtype == VALMOD_F32 ? 4 : 8;
  const void* sub_series = (const char*)d_series + (size_t)Ls.series * esz;
  valmod_outputs so;
  memset(&so, 0, sizeof(so));
  struct Cand {
    int hmul;
    int32_t R;
    int K;
    int32_t p;
    bool no_heaps;
  };
  // time one candidate on lengths [lo, hi] of the tuned series (ms, -1 if it does not fit)
  auto time_run = [&](const Cand& c, int32_t lo, int32_t hi, int32_t path, double* ms) -> valmod_status {
    valmod_config sc = P->cfg;
    const int64_t n1 = Ls.n;
    sc.num_series = 1;
    sc.n = &n1;
    sc.l_min = &lo;
    sc.l_max = &hi;
    sc.path = path;
    sc.lanes = 1;
    sc.graph = 0;
    sc.refresh_R = c.R;
    sc.p = c.p;
    sc.m_discords = 1;  // what is timed is the pass geometry and the partial profiles
    sc.mset_radius = 0.0;
    sc.mode = VALMOD_MODE_EXACT;
    valmod_plan_t sub = nullptr;
    valmod_status st = valmod_plan(&sc, &sub);
    if (st != VALMOD_OK) return st;
    sub->tune_hmul = c.hmul;
    sub->tune_K = c.K;
    build_layout(sub);
    *ms = -1.0;
    if (sub->ws_total <= P->ws_total) {
      st = valmod_run(sub, sub_series, d_ws, &so, stream);
      if (st == VALMOD_OK) st = valmod_run_status(sub, stream);
      const auto t0 = std::chrono::steady_clock::now();
      if (st == VALMOD_OK) st = valmod_run(sub, sub_series, d_ws, &so, stream);
      if (st == VALMOD_OK) st = valmod_run_status(sub, stream);
      *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    valmod_plan_free(sub);
    return st;
  };
  Cand best{P->tune_hmul, P->tune_R, P->tune_K, P->cfg.p, P->tune_no_heaps};
  // stage 1: pass geometry
  std::vector<Cand> cand;
  const bool k_fixed = env_int(fp32 ? "VALMOD_PASS_K32" : "VALMOD_PASS_K", 0) != 0;
  if (fp32) {
    if (P->cfg.refresh_R <= 0)
      for (int32_t R : {256, 512, 1024})
        for (int K : {8, 4})
          if (K == 8 || !k_fixed) cand.push_back({1, R, k_fixed ? 0 : K, P->cfg.p, P->tune_no_heaps});
  } else if (env_int("VALMOD_PASS_H", 0) == 0) {
    for (int h : {1, 2, 4}) cand.push_back({h, 0, 0, P->cfg.p, P->tune_no_heaps});
  }
  const int32_t T = (int32_t)std::min<int64_t>(3, Ls.nlen);
  const int32_t lo_a = Ls.l_min, lo_b = std::max<int32_t>(Ls.l_min, Ls.l_max - T + 1);
  if (cand.size() >= 2) {
    double best_ms = -1.0;
    for (const Cand& c : cand) {
      double ms_a = 0.0, ms_b = 0.0;
      valmod_status st = time_run(c, lo_a, lo_a + T - 1, VALMOD_PATH_FULL, &ms_a);
      if (st == VALMOD_OK && ms_a >= 0.0 && lo_b > lo_a) st = time_run(c, lo_b, lo_b + T - 1, VALMOD_PATH_FULL, &ms_b);
      if (st != VALMOD_OK) return st;
      if (ms_a < 0.0 || ms_b < 0.0) continue;  // does not fit the workspace
      const double ms = ms_a + ms_b;
      if (best_ms < 0.0 || ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  // stage 2: p (exact mode with partial profiles), and no partial profiles at all
  // (the lower bound may fail right after the first length, as on periodic data;
  // the outputs are the same)
  const bool heaps = P->cfg.mode == VALMOD_MODE_EXACT && P->cfg.path != VALMOD_PATH_FULL && P->cfg.m_discords <= 1 &&
                     !P->cfg.graph && Ls.nlen >= 2;
  if (heaps) {
    const int32_t T2 = (int32_t)std::min<int64_t>(4, Ls.nlen);
    double best_ms = -1.0;
    Cand keep = best;
    std::vector<int32_t> pcs;
    for (int32_t pc : {P->cfg.p, P->cfg.p / 2, P->cfg.p / 4})
      if (pc >= 1 && std::find(pcs.begin(), pcs.end(), pc) == pcs.end()) pcs.push_back(pc);
    pcs.push_back(0);  // partial profiles off
    for (int32_t pc : pcs) {
      Cand c = keep;
      c.p = pc > 0 ? pc : keep.p;
      c.no_heaps = pc == 0;
      double ms = 0.0;
      const valmod_status st =
          time_run(c, Ls.l_min, Ls.l_min + T2 - 1, c.no_heaps ? (int32_t)VALMOD_PATH_FULL : P->cfg.path, &ms);
      if (st != VALMOD_OK) return st;
      if (ms < 0.0) continue;
      if (best_ms < 0.0 || ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  const Cand old{P->tune_hmul, P->tune_R, P->tune_K, P->cfg.p, P->tune_no_heaps};
  const int64_t old_cap = P->cap;
  const size_t old_total = P->ws_total;
  auto apply = [&](const Cand& c) {
    P->tune_hmul = c.hmul;
    P->tune_R = c.R;
    P->tune_K = c.K;
    P->tune_no_heaps = c.no_heaps;
    P->cfg.p = c.p;
    P->cap = 8 * (int64_t)c.p < 64 ? 64 : (8 * (int64_t)c.p > 512 ? 512 : 8 * (int64_t)c.p);
    const int cap_env = env_int("VALMOD_COLLECT_CAP", 0);
    if (cap_env > 0) P->cap = cap_env < 512 ? cap_env : 512;
    build_layout(P);
  };
  apply(best);
  if (P->ws_total > old_total) {  // never needs more workspace than the caller holds
    apply(old);
    P->cap = old_cap;
    build_layout(P);
  }
  if (P->exec) {  // a captured run used the old geometry
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(P->cfg.device) == hipSuccess) {
      (void)hipGraphExecDestroy(P->exec);
      (void)hipSetDevice(prev);
    }
    P->exec = nullptr;
  }
  if (chosen) {
    chosen[0] = (int32_t)P->geom[sbest].H;
    chosen[1] = P->geom[sbest].K;
    chosen[2] = P->tune_no_heaps ? 0 : P->cfg.p;
  }
  return VALMOD_OK;
}

extern "C" double valmod_rounding_bound(int32_t precision, int64_t H, int32_t L, double phi, double psi, double xi) {
  if (H < 1 || L < 1 || !(phi >= 0.0) || !(psi >= 0.0) || !(xi >= 0.0)) return NAN;
  if (precision == VALMOD_PREC_FP32_REFRESH)
    return recurrence_bound(kEps32, (double)H, phi, psi, xi, L) + kFilter32;
  if (precision == VALMOD_PREC_FP64) return recurrence_bound(kEps64, (double)H, phi, psi, xi, L);
  return NAN;
}
