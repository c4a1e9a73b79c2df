// C ABI of the GMM-Tree library: handles, workspace layout, level planning
// and the launch sequence of tree construction and registration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <array>
#include <mutex>
#include <vector>

#include "../../include/hgmm.h"
#include "hgmm_dev.h"
#include "hgmm_host.h"
#include "hgmm_internal.h"

using namespace hgmm;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hgmm_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(HGMM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define HIP_LAUNCHED()                                                                                 \
  do {                                                                                                 \
    hipError_t e_ = hipGetLastError();                                                                 \
    if (e_ != hipSuccess) return fail(HGMM_EHIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

static int64_t level_off(int l) { return (((int64_t)1 << (3 * (l + 1))) - 8) / 7; }
static int64_t level_nodes(int l) { return (int64_t)1 << (3 * (l + 1)); }
static int64_t tree_nodes(int L) { return level_off(L); }

// ---------------------------------------------------------------------------
// forest handle
// ---------------------------------------------------------------------------

struct TreeHost {
  int levels;
  int64_t n_points;
  int64_t node_base;
  int64_t point_off;
  int64_t label_base;
};

struct hgmm_forest_s {
  int device = 0;
  std::vector<TreeHost> trees;
  // host planner's scratch (jobs of a level, a tiled job's slot), kept with
  // the handle so that a construction reuses their memory
  std::vector<Job> plan_jobs;
  std::vector<int> plan_slot;
  TreeDev* d_trees = nullptr;
  size_t cap_trees = 0;
  NodeD* d_nodes = nullptr;
  NodeF* d_tab = nullptr;
  int64_t cap_nodes = 0;
  int64_t cap_tab = 0;
  int32_t* d_labels = nullptr;
  int64_t cap_labels = 0;
  bool has_labels = false;
  char* h_stage = nullptr;
  size_t cap_stage = 0;
  // side streams (default priority) on which the block-class EM launches of a
  // level run concurrently with the tiled iterations on the caller's stream
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[3] = {nullptr, nullptr, nullptr};
  // registration chunk graph (reg_graph = 1): capture stream, fork/join
  // events, the instantiated graph and the launch arguments it was built for
  hipStream_t gstream = nullptr;
  hipEvent_t ev_g0 = nullptr, ev_g1 = nullptr;
  hipGraphExec_t reg_exec = nullptr;
  std::vector<uint64_t> reg_key;
  // construction graph (build_graph = 1): every level planned on the device,
  // all launches of a construction in one graph, cached for the same shapes
  // (build_graph = 2: the same launches issued on the stream, no graph)
  hipGraphExec_t bld_exec = nullptr;
  std::vector<uint64_t> bld_key;
  // per-level work counts of the last host-planned construction (njobs,
  // ntiles, nbig, jobs per class) and the shape they belong to: the graph's
  // fixed grids are sized from them
  std::vector<std::array<int, 7>> hint;
  std::vector<uint64_t> hint_key;
  int64_t n_graph_replays = 0, n_graph_captures = 0, n_host_builds = 0;
  int64_t total_nodes() const {
    int64_t s = 0;
    for (auto& t : trees) s += tree_nodes(t.levels);
    return s;
  }
};

int hgmm_forest_size(const hgmm_forest_s* f) { return (int)f->trees.size(); }
TreeDev* hgmm_forest_trees(hgmm_forest_s* f) { return f->d_trees; }
NodeD* hgmm_forest_nodes(hgmm_forest_s* f) { return f->d_nodes; }

static void free_forest(hgmm_forest_s* f) {
  if (!f) return;
  if (f->d_trees) (void)hipFree(f->d_trees);
  if (f->d_nodes) (void)hipFree(f->d_nodes);
  if (f->d_tab) (void)hipFree(f->d_tab);
  if (f->d_labels) (void)hipFree(f->d_labels);
  if (f->h_stage) (void)hipHostFree(f->h_stage);
  for (int c = 0; c < 3; ++c) {
    if (f->side[c]) (void)hipStreamDestroy(f->side[c]);
    if (f->ev_join[c]) (void)hipEventDestroy(f->ev_join[c]);
  }
  if (f->ev_fork) (void)hipEventDestroy(f->ev_fork);
  if (f->reg_exec) (void)hipGraphExecDestroy(f->reg_exec);
  if (f->bld_exec) (void)hipGraphExecDestroy(f->bld_exec);
  if (f->gstream) (void)hipStreamDestroy(f->gstream);
  if (f->ev_g0) (void)hipEventDestroy(f->ev_g0);
  if (f->ev_g1) (void)hipEventDestroy(f->ev_g1);
  delete f;
}

static int ensure_graph_stream(hgmm_forest_s* f) {
  if (f->gstream) return HGMM_OK;
  if (hipStreamCreateWithFlags(&f->gstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&f->ev_g0, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&f->ev_g1, hipEventDisableTiming) != hipSuccess)
    return fail(HGMM_EHIP, "graph stream creation failed");
  return HGMM_OK;
}

static int ensure_side_streams(hgmm_forest_s* f) {
  if (f->ev_fork) return HGMM_OK;
  for (int c = 0; c < 3; ++c) {
    if (hipStreamCreateWithFlags(&f->side[c], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&f->ev_join[c], hipEventDisableTiming) != hipSuccess)
      return fail(HGMM_EHIP, "side stream creation failed");
  }
  if (hipEventCreateWithFlags(&f->ev_fork, hipEventDisableTiming) != hipSuccess)
    return fail(HGMM_EHIP, "event creation failed");
  return HGMM_OK;
}

template <typename T>
static int grow_dev(T*& p, int64_t& cap, int64_t need) {
  if (need <= cap && p) return HGMM_OK;
  if (p) { (void)hipFree(p); p = nullptr; }
  cap = 0;
  if (hipMalloc((void**)&p, sizeof(T) * (size_t)std::max<int64_t>(need, 1)) != hipSuccess)
    return fail(HGMM_ENOMEM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * need));
  cap = need;
  return HGMM_OK;
}

static int grow_stage(hgmm_forest_s* f, size_t need) {
  if (need <= f->cap_stage && f->h_stage) return HGMM_OK;
  if (f->h_stage) { (void)hipHostFree(f->h_stage); f->h_stage = nullptr; }
  f->cap_stage = 0;
  size_t sz = std::max<size_t>(need, 1 << 16);
  if (hipHostMalloc((void**)&f->h_stage, sz, hipHostMallocDefault) != hipSuccess)
    return fail(HGMM_ENOMEM, "pinned host allocation of %zu bytes failed", sz);
  f->cap_stage = sz;
  return HGMM_OK;
}

// Lays out `trees` (levels and point counts already set) and sizes the device
// arrays of the forest.
static int setup_forest(hgmm_forest_s* f) {
  int64_t nb = 0, lb = 0, pb = 0;
  for (auto& t : f->trees) {
    t.node_base = nb;
    t.label_base = lb;
    t.point_off = pb;
    nb += tree_nodes(t.levels);
    lb += (int64_t)t.levels * t.n_points;
    pb += t.n_points;
  }
  int64_t ct = (int64_t)f->cap_trees;
  int st = grow_dev(f->d_trees, ct, (int64_t)f->trees.size());
  f->cap_trees = (size_t)ct;
  if (st) return st;
  if ((st = grow_dev(f->d_nodes, f->cap_nodes, nb))) return st;
  if ((st = grow_dev(f->d_tab, f->cap_tab, nb))) return st;
  if ((st = grow_dev(f->d_labels, f->cap_labels, std::max<int64_t>(lb, 1)))) return st;
  return HGMM_OK;
}

// ---------------------------------------------------------------------------
// workspace layouts
// ---------------------------------------------------------------------------

static size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

struct BuildLayout {
  size_t pts[2], perm[2], child, tiles, tile_ids, job_ids, jobs, partials, partials2, chbuf, frames, tile_counts,
      tile_base, lvl_info, level_trees, plans, total;
  int64_t max_tiles, max_jobs, max_lvl;
};

static BuildLayout build_layout(int64_t n_total, int64_t max_jobs, int64_t max_lvl, int B, int Lmax) {
  BuildLayout L;
  L.max_jobs = std::max<int64_t>(max_jobs, 1);
  L.max_tiles = n_total / 64 + L.max_jobs + 1;
  L.max_lvl = std::max<int64_t>(max_lvl, 8);
  size_t o = 0;
  for (int k = 0; k < 2; ++k) { L.pts[k] = o; o = align_up(o + sizeof(float) * 3 * (size_t)n_total); }
  for (int k = 0; k < 2; ++k) { L.perm[k] = o; o = align_up(o + sizeof(int) * (size_t)n_total); }
  L.child = o; o = align_up(o + (size_t)n_total);
  // level plan region [tiles, partials): holds the packed jobs | tiles | tile
  // ids | job ids of one level (at most these four maxima)
  L.tiles = o; o = align_up(o + sizeof(Tile) * (size_t)L.max_tiles);
  L.tile_ids = o; o = align_up(o + sizeof(int) * (size_t)L.max_tiles);
  L.job_ids = o; o = align_up(o + sizeof(int) * (size_t)L.max_jobs);
  L.jobs = o; o = align_up(o + sizeof(Job) * (size_t)L.max_jobs);
  L.partials = o; o = align_up(o + sizeof(double) * 80 * (size_t)L.max_tiles);
  L.partials2 = o; o = align_up(o + sizeof(double) * 80 * (size_t)L.max_tiles);
  L.chbuf = o; o = align_up(o + sizeof(NodeF) * 8 * (size_t)L.max_jobs);
  L.frames = o; o = align_up(o + kFrameBytes * (size_t)L.max_jobs);
  L.tile_counts = o; o = align_up(o + sizeof(int) * 9 * (size_t)L.max_tiles);
  L.tile_base = o; o = align_up(o + sizeof(int) * 9 * (size_t)L.max_tiles);
  L.lvl_info = o; o = align_up(o + sizeof(int2) * (size_t)L.max_lvl);
  // construction planned on the device: the trees of every level and the
  // level plans (PlanField ints)
  L.level_trees = o; o = align_up(o + sizeof(LevelTree) * (size_t)std::max(B, 1) * (size_t)std::max(Lmax, 1));
  L.plans = o; o = align_up(o + sizeof(int) * PL_SIZE * (size_t)std::max(Lmax, 1));
  L.total = o;
  return L;
}

struct RegLayout {
  size_t bins, state, nmov, tiles, out, fbins, regf, ptiles, active, pose, keys, keys2, vals, perm, sxyz, sort_temp,
      flatf, total;
  size_t sort_temp_bytes;
  int64_t max_tiles;
};

static RegLayout reg_layout(int64_t n_total, int64_t nodes, int npairs) {
  RegLayout L;
  L.max_tiles = n_total / 256 + npairs + 1;
  size_t o = 0;
  L.bins = o; o = align_up(o + sizeof(double) * 6 * (size_t)std::max<int64_t>(nodes, 1));
  L.fbins = o; o = align_up(o + sizeof(FixBin) * (size_t)std::max<int64_t>(nodes, 1));  // fixed-point moments
  L.regf = o; o = align_up(o + sizeof(NodeR) * (size_t)std::max<int64_t>(nodes, 1));   // descent scoring records
  // per-pair inputs uploaded together: tile ranges | point counts | start
  // poses (12 doubles: R row-major, t) | active flags
  L.ptiles = o; o = align_up(o + sizeof(int2) * (size_t)npairs);
  L.nmov = o; o = align_up(o + sizeof(int64_t) * (size_t)npairs);
  L.pose = o; o = align_up(o + sizeof(double) * 12 * (size_t)npairs);
  L.active = o; o = align_up(o + sizeof(int) * (size_t)npairs);
  L.state = o; o = align_up(o + sizeof(PoseState) * (size_t)npairs);
  L.tiles = o; o = align_up(o + sizeof(Tile) * (size_t)L.max_tiles);
  L.out = o; o = align_up(o + sizeof(double) * 28 * (size_t)npairs + sizeof(double) * 12 * npairs);
  // Morton ordering of the moving points (reg_sort)
  L.keys = o; o = align_up(o + sizeof(uint64_t) * (size_t)n_total);
  L.keys2 = o; o = align_up(o + sizeof(uint64_t) * (size_t)n_total);
  L.vals = o; o = align_up(o + sizeof(int) * (size_t)n_total);
  L.perm = o; o = align_up(o + sizeof(int) * (size_t)n_total);
  L.sxyz = o; o = align_up(o + sizeof(float) * 3 * (size_t)n_total);
  L.sort_temp_bytes = sort_temp_bytes(n_total, npairs);
  L.sort_temp = o; o = align_up(o + L.sort_temp_bytes);
  // scoring records with global weights (single-level E-step)
  L.flatf = o; o = align_up(o + sizeof(NodeR) * (size_t)std::max<int64_t>(nodes, 1));  // single-level records
  L.total = o;
  return L;
}

static int64_t max_jobs_for(const std::vector<TreeHost>& trees) {
  int64_t m = 0;
  int Lmax = 0;
  for (auto& t : trees) Lmax = std::max(Lmax, t.levels);
  for (int l = 0; l < Lmax; ++l) {
    int64_t s = 0;
    for (auto& t : trees)
      if (t.levels > l) s += (l == 0) ? 1 : level_nodes(l - 1);
    m = std::max(m, s);
  }
  return m;
}

static int64_t max_lvl_for(const std::vector<TreeHost>& trees) {
  int64_t m = 0;
  int Lmax = 0;
  for (auto& t : trees) Lmax = std::max(Lmax, t.levels);
  for (int l = 0; l < Lmax; ++l) {
    int64_t s = 0;
    for (auto& t : trees)
      if (t.levels > l) s += level_nodes(l);
    m = std::max(m, s);
  }
  return m;
}

// ---------------------------------------------------------------------------
// launch shapes (process wide; see hgmm_tuning)
// ---------------------------------------------------------------------------

static hgmm_tuning g_tune = {256, 2048, 8192, 1024, 1024, 4096, 512, 4, 0, 0, 256, 2, 0, 0, 1024};

extern "C" int hgmm_set_tuning(const hgmm_tuning* t) {
  if (!t) return fail(HGMM_EINVAL, "null tuning");
  const int lim = 1 << 20;
  if (!(0 <= t->block64_max && t->block64_max <= t->block256_max && t->block256_max <= t->block512_max &&
        t->block512_max <= lim))
    return fail(HGMM_EINVAL, "block thresholds must satisfy 0 <= b64 <= b256 <= b512 <= 2^20");
  if (!(64 <= t->min_tile && t->min_tile <= t->max_tile && t->max_tile <= lim && t->target_tiles >= 1))
    return fail(HGMM_EINVAL, "tile sizes must satisfy 64 <= min_tile <= max_tile <= 2^20, target_tiles >= 1");
  if (!(256 <= t->reg_tile && t->reg_tile <= lim && 1 <= t->reg_chunk && t->reg_chunk <= 64))
    return fail(HGMM_EINVAL, "reg_tile must be in [256, 2^20] and reg_chunk in [1, 64]");
  if (t->reg_graph != 0 && t->reg_graph != 1) return fail(HGMM_EINVAL, "reg_graph must be 0 or 1");
  if (t->reg_sort != 0 && t->reg_sort != 1) return fail(HGMM_EINVAL, "reg_sort must be 0 or 1");
  if (t->tile_threads != 256 && t->tile_threads != 512 && t->tile_threads != 1024)
    return fail(HGMM_EINVAL, "tile_threads must be 256, 512 or 1024");
  if (t->reg_lds_levels != 2 && t->reg_lds_levels != 3) return fail(HGMM_EINVAL, "reg_lds_levels must be 2 or 3");
  if (t->build_graph < 0 || t->build_graph > 2) return fail(HGMM_EINVAL, "build_graph must be 0, 1 or 2");
  if (t->reg_atomics != 0 && t->reg_atomics != 1) return fail(HGMM_EINVAL, "reg_atomics must be 0 or 1");
  if (t->fold_tiles < 0) return fail(HGMM_EINVAL, "fold_tiles must be >= 0");
  g_tune = *t;
  g_tune.min_tile = (t->min_tile + 63) / 64 * 64;
  g_tune.max_tile = (t->max_tile + 63) / 64 * 64;
  g_tune.reg_tile = (t->reg_tile + 255) / 256 * 256;
  return HGMM_OK;
}

extern "C" int hgmm_get_tuning(hgmm_tuning* t) {
  if (!t) return fail(HGMM_EINVAL, "null tuning");
  *t = g_tune;
  return HGMM_OK;
}

static int tile_points(int64_t level_points) {
  int64_t t = level_points / std::max(1, g_tune.target_tiles);
  t = (t + 63) / 64 * 64;
  t = std::max<int64_t>(t, g_tune.min_tile);
  t = std::min<int64_t>(t, g_tune.max_tile);
  return (int)t;
}

// ---------------------------------------------------------------------------
// optional event timing of the kernel launches (benchmark instrumentation)
// ---------------------------------------------------------------------------

enum ProfKind { PK_EM_TILE = 0, PK_EM_BLOCK, PK_PARTITION, PK_SCATTER, PK_DESCEND, PK_NORMAL, PK_ROOT, PK_EM_MSTEP,
                PK_FLAT, PK_SOFT, PK_COUNT };

struct ProfPending {
  int kind;
  double units;
  hipEvent_t a, b;
  int tag;    // registration iteration of a descend/normal launch, -1 otherwise
  int wslot;  // device work-counter slot of a descend launch, -1 otherwise
};

constexpr int kProfWorkSlots = 8192;

struct ProfState {
  bool on = false;
  double ms[PK_COUNT] = {0};
  int64_t launches[PK_COUNT] = {0};
  double units[PK_COUNT] = {0};
  double points[PK_COUNT] = {0};  // device-counted points processed (descend)
  double levels[PK_COUNT] = {0};  // device-counted levels those points scored (descend)
  std::vector<hipEvent_t> pool;
  std::vector<ProfPending> pending;
  unsigned long long* d_work = nullptr;  // 2 counters per slot, allocated when profiling starts
  int next_slot = 0;
};
static ProfState g_prof;

static hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct ProfScope {
  ProfPending p;
  hipStream_t s;
  bool on;
  ProfScope(int kind, double units, hipStream_t st, int tag = -1, bool enable = true)
      : s(st), on(g_prof.on && enable) {
    p.wslot = -1;
    if (!on) return;
    p.kind = kind; p.units = units; p.tag = tag;
    p.a = prof_event(); p.b = prof_event();
    (void)hipEventRecord(p.a, s);
  }
  // device counters of the points this launch processes and the levels they
  // score (zeroed; nullptr when not profiling or out of slots)
  unsigned long long* work_slot() {
    if (!on || !g_prof.d_work || g_prof.next_slot >= kProfWorkSlots) return nullptr;
    p.wslot = g_prof.next_slot++;
    return g_prof.d_work + 2 * p.wslot;
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(p.b, s);
    g_prof.pending.push_back(p);
  }
};

// Folds the timed launches into the totals (call after the stream was
// synchronised).  Every launch counts, also those queued after every pair
// had converged (they exit at once and add no work), so that launch counts
// and average durations are those a kernel trace of the same run shows.
static void prof_collect(int iters_done = 1 << 30) {
  (void)iters_done;
  std::vector<unsigned long long> work;
  if (g_prof.d_work && g_prof.next_slot > 0) {
    work.resize(2 * (size_t)g_prof.next_slot);
    if (hipMemcpy(work.data(), g_prof.d_work, sizeof(unsigned long long) * work.size(), hipMemcpyDeviceToHost) !=
        hipSuccess)
      work.clear();
    (void)hipMemset(g_prof.d_work, 0, sizeof(unsigned long long) * 2 * kProfWorkSlots);
    g_prof.next_slot = 0;
  }
  for (auto& p : g_prof.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_prof.ms[p.kind] += ms;
      g_prof.launches[p.kind] += 1;
      g_prof.units[p.kind] += p.units;
      if (p.wslot >= 0 && (size_t)(2 * p.wslot + 1) < work.size()) {
        g_prof.points[p.kind] += (double)work[2 * p.wslot];
        g_prof.levels[p.kind] += (double)work[2 * p.wslot + 1];
      }
    }
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
}

extern "C" int hgmm_profile(int enable) {
  if (enable && !g_prof.d_work) {
    if (hipMalloc((void**)&g_prof.d_work, sizeof(unsigned long long) * 2 * kProfWorkSlots) != hipSuccess)
      return fail(HGMM_ENOMEM, "profiling counters could not be allocated");
    if (hipMemset(g_prof.d_work, 0, sizeof(unsigned long long) * 2 * kProfWorkSlots) != hipSuccess)
      return fail(HGMM_EHIP, "profiling counters could not be cleared");
    g_prof.next_slot = 0;
  }
  g_prof.on = enable != 0;
  return HGMM_OK;
}

extern "C" void hgmm_profile_reset(void) {
  for (int k = 0; k < PK_COUNT; ++k) {
    g_prof.ms[k] = 0; g_prof.launches[k] = 0; g_prof.units[k] = 0; g_prof.points[k] = 0; g_prof.levels[k] = 0;
  }
}

extern "C" int hgmm_profile_work(int kind, double* points, double* levels) {
  if (kind < 0 || kind >= PK_COUNT) return fail(HGMM_EINVAL, "profile kind %d out of range", kind);
  if (points) *points = g_prof.points[kind];
  if (levels) *levels = g_prof.levels[kind];
  return HGMM_OK;
}

extern "C" int hgmm_profile_read(int kind, double* total_ms, int64_t* launches, double* units) {
  if (kind < 0 || kind >= PK_COUNT) return fail(HGMM_EINVAL, "profile kind %d out of range", kind);
  if (total_ms) *total_ms = g_prof.ms[kind];
  if (launches) *launches = g_prof.launches[kind];
  if (units) *units = g_prof.units[kind];
  return HGMM_OK;
}

// ---------------------------------------------------------------------------
// construction
// ---------------------------------------------------------------------------

struct BuildInput {
  const float* xs;
  const float* ys;
  const float* zs;
};

// The shape of a construction: clouds (sizes, depths), parameters and launch
// shapes; a construction graph, and the work counts that size its grids,
// belong to one shape.
static std::vector<uint64_t> build_shape_key(const hgmm_forest_s* f, const hgmm_build_params& p) {
  uint64_t eps_bits, mm_bits;
  memcpy(&eps_bits, &p.reg_eps, 8);
  memcpy(&mm_bits, &p.min_mass, 8);
  std::vector<uint64_t> key = {(uint64_t)f->trees.size(), (uint64_t)p.build_iters, eps_bits, mm_bits};
  // every launch shape except build_graph itself (a host-planned construction
  // records the counts a later graph construction uses)
  hgmm_tuning tu = g_tune;
  tu.build_graph = 0;
  const int32_t* tv = (const int32_t*)&tu;
  for (size_t k = 0; k < sizeof(hgmm_tuning) / sizeof(int32_t); ++k) key.push_back((uint64_t)(uint32_t)tv[k]);
  for (auto& t : f->trees) key.push_back(((uint64_t)t.levels << 40) | (uint64_t)t.n_points);
  return key;
}

static int run_build(hgmm_forest_s* f, BuildInput in, const hgmm_build_params& p, char* ws, size_t ws_bytes,
                     hipStream_t s) {
  const int B = (int)f->trees.size();
  int64_t n_total = 0;
  int Lmax = 0;
  for (auto& t : f->trees) { n_total += t.n_points; Lmax = std::max(Lmax, t.levels); }
  BuildLayout Ly = build_layout(n_total, max_jobs_for(f->trees), max_lvl_for(f->trees), B, Lmax);
  if (ws_bytes < Ly.total) return fail(HGMM_EINVAL, "build workspace too small: %zu < %zu", ws_bytes, Ly.total);
  float* pts[2] = {(float*)(ws + Ly.pts[0]), (float*)(ws + Ly.pts[1])};
  int* perm[2] = {(int*)(ws + Ly.perm[0]), (int*)(ws + Ly.perm[1])};
  uint8_t* child = (uint8_t*)(ws + Ly.child);
  // the level plan (jobs | tiles | tile ids | job ids) is packed into the
  // region [Ly.tiles, Ly.partials) and uploaded with one copy per level
  char* d_plan = ws + Ly.tiles;
  Tile* d_tiles = nullptr;
  int* d_tile_ids = nullptr;
  int* d_job_ids = nullptr;
  Job* d_jobs = nullptr;
  double* d_partials = (double*)(ws + Ly.partials);
  double* d_part[2] = {d_partials, (double*)(ws + Ly.partials2)};
  // children (8 per tiled job) and the next E-step's frame (kFrameBytes per
  // tiled job) of the tiled jobs between iterations; with the fold inside
  // the tile blocks the two regions are the children's ping-pong buffers
  NodeF* d_ch = (NodeF*)(ws + Ly.chbuf);
  void* d_frames = ws + Ly.frames;
  int* d_tile_counts = (int*)(ws + Ly.tile_counts);
  int* d_tile_base = (int*)(ws + Ly.tile_base);
  int2* d_lvl = (int2*)(ws + Ly.lvl_info);

  // staging: trees | jobs | tiles | tile ids | job ids | level info
  size_t st_trees = 0;
  size_t st_jobs = align_up(st_trees + sizeof(TreeDev) * 2 * B);
  size_t st_tiles = align_up(st_jobs + sizeof(Job) * Ly.max_jobs);
  size_t st_tids = align_up(st_tiles + sizeof(Tile) * Ly.max_tiles);
  size_t st_jids = align_up(st_tids + sizeof(int) * Ly.max_tiles);
  size_t st_lvl = align_up(st_jids + sizeof(int) * Ly.max_jobs);
  size_t st_end = align_up(st_lvl + sizeof(int2) * Ly.max_lvl);
  int rc = grow_stage(f, st_end);
  if (rc) return rc;
  char* H = f->h_stage;
  TreeDev* h_trees = (TreeDev*)(H + st_trees);
  Job* h_jobs = (Job*)(H + st_jobs);
  Tile* h_tiles = (Tile*)(H + st_tiles);
  int* h_tids = (int*)(H + st_tids);
  int* h_jids = (int*)(H + st_jids);
  int2* h_lvl = (int2*)(H + st_lvl);

  for (int b = 0; b < B; ++b) {
    TreeDev& T = h_trees[b];
    memset(&T, 0, sizeof(T));
    T.node_base = f->trees[b].node_base;
    T.point_off = f->trees[b].point_off;
    T.label_base = f->trees[b].label_base;
    T.levels = f->trees[b].levels;
    T.n_points = (int32_t)f->trees[b].n_points;
  }
  HIP_TRY(hipMemcpyAsync(f->d_trees, h_trees, sizeof(TreeDev) * B, hipMemcpyHostToDevice, s));
  const int64_t nodes_total = f->total_nodes();
  launch_fill_u32(f->d_nodes, 0u, (int64_t)(sizeof(NodeD) / 4) * nodes_total, s);
  launch_fill_u32(f->d_tab, 0u, (int64_t)(sizeof(NodeF) / 4) * nodes_total, s);
  int64_t nlab = 0;
  for (auto& t : f->trees) nlab += (int64_t)t.levels * t.n_points;
  launch_fill_u32(f->d_labels, 0xFFFFFFFFu, nlab, s);
  HIP_LAUNCHED();

  // level-compact bases: lvl_base[l][b]
  std::vector<std::vector<int64_t>> lvl_base(Lmax, std::vector<int64_t>(B, -1));
  std::vector<int64_t> lvl_size(Lmax, 0);
  for (int l = 0; l < Lmax; ++l)
    for (int b = 0; b < B; ++b)
      if (f->trees[b].levels > l) { lvl_base[l][b] = lvl_size[l]; lvl_size[l] += level_nodes(l); }

  const float* cx = in.xs;
  const float* cy = in.ys;
  const float* cz = in.zs;
  const int* cperm = nullptr;
  int ping = 0;
  std::vector<Job>& jobs = f->plan_jobs;
  jobs.reserve((size_t)Ly.max_jobs);

  std::vector<std::array<int, 7>> hint((size_t)Lmax, std::array<int, 7>{0, 0, 0, 0, 0, 0, 0});
  for (int l = 0; l < Lmax; ++l) {
    // ---- plan the jobs of level l (parents at level l-1, roots at level 0)
    jobs.clear();
    int64_t level_points = 0;
    if (l == 0) {
      for (int b = 0; b < B; ++b) {
        const TreeHost& t = f->trees[b];
        Job j;
        j.start = (int32_t)t.point_off;
        j.count = (int32_t)t.n_points;
        j.parent = -1;
        j.child_base = (int32_t)t.node_base;
        j.child_lvl = (int32_t)lvl_base[0][b];
        j.tree = b;
        jobs.push_back(j);
        level_points += t.n_points;
      }
    } else {
      for (int b = 0; b < B; ++b) {
        const TreeHost& t = f->trees[b];
        if (t.levels <= l) continue;
        const int64_t pb = lvl_base[l - 1][b];
        const int64_t np = level_nodes(l - 1);
        for (int64_t k = 0; k < np; ++k) {
          const int2 info = h_lvl[pb + k];
          if (info.y <= 0) continue;
          Job j;
          j.start = info.x;
          j.count = info.y;
          j.parent = (int32_t)(t.node_base + level_off(l - 1) + k);
          j.child_base = (int32_t)(t.node_base + level_off(l) + 8 * k);
          j.child_lvl = (int32_t)(lvl_base[l][b] + 8 * k);
          j.tree = b;
          jobs.push_back(j);
          level_points += info.y;
        }
      }
    }
    const int njobs = (int)jobs.size();
    if (njobs == 0) break;
    const int tpts = tile_points(level_points);
    // job classes: 0..2 one block of 64 / 256 / 512 threads per job for all
    // iterations, 3 tiled; h_jids lists the jobs class by class
    int ntiles = 0, nbig = 0;
    int cls_n[4] = {0, 0, 0, 0}, cls_off[5] = {0, 0, 0, 0, 0};
    int64_t cls_points[4] = {0, 0, 0, 0};
    auto job_class = [](int count) {
      return count <= g_tune.block64_max ? 0 : count <= g_tune.block256_max ? 1 : count <= g_tune.block512_max ? 2 : 3;
    };
    for (int j = 0; j < njobs; ++j) { cls_n[job_class(jobs[j].count)] += 1; cls_points[job_class(jobs[j].count)] += jobs[j].count; }
    for (int c = 0; c < 4; ++c) cls_off[c + 1] = cls_off[c] + cls_n[c];
    // slot of each tiled job among the tiled jobs (its child records in the
    // ping-pong buffers and its block in the final M-step)
    std::vector<int>& slot_of = f->plan_slot;
    slot_of.assign((size_t)njobs, 0);
    {
      int fill[4] = {cls_off[0], cls_off[1], cls_off[2], cls_off[3]};
      for (int j = 0; j < njobs; ++j) {
        const int c = job_class(jobs[j].count);
        if (c == 3) slot_of[(size_t)j] = fill[3] - cls_off[3];
        h_jids[fill[c]++] = j;
      }
    }
    for (int j = 0; j < njobs; ++j) {
      Job& jb = jobs[j];
      jb.tile_first = ntiles;
      jb.ntiles = (jb.count + tpts - 1) / tpts;
      const bool tiled = job_class(jb.count) == 3;
      for (int t = 0; t < jb.ntiles; ++t) {
        Tile& T = h_tiles[ntiles];
        T.start = jb.start + t * tpts;
        T.end = std::min(jb.start + jb.count, T.start + tpts);
        T.job = j;
        T.pad = tiled ? slot_of[(size_t)j] : 0;
        if (tiled) h_tids[nbig++] = ntiles;
        ++ntiles;
      }
      h_jobs[j] = jb;
    }
    const int nbigjobs = cls_n[3];
    if (ntiles > Ly.max_tiles || njobs > Ly.max_jobs) return fail(HGMM_EINVAL, "internal: tile plan overflow");
    hint[l] = {njobs, ntiles, nbig, cls_n[0], cls_n[1], cls_n[2], cls_n[3]};
    {
      // pack the plan behind the jobs in the staging buffer (every table moves
      // to a lower or equal offset, in order, so nothing is overwritten before
      // it is moved) and upload it with one copy; the previous level's copy
      // has completed (the stream was synchronised for the level sizes)
      const size_t o_tiles = align_up(sizeof(Job) * (size_t)njobs);
      const size_t o_tids = align_up(o_tiles + sizeof(Tile) * (size_t)ntiles);
      const size_t o_jids = align_up(o_tids + sizeof(int) * (size_t)nbig);
      const size_t o_end = o_jids + sizeof(int) * (size_t)njobs;
      char* hp = (char*)h_jobs;
      memmove(hp + o_tiles, h_tiles, sizeof(Tile) * (size_t)ntiles);
      memmove(hp + o_tids, h_tids, sizeof(int) * (size_t)nbig);
      memmove(hp + o_jids, h_jids, sizeof(int) * (size_t)njobs);
      HIP_TRY(hipMemcpyAsync(d_plan, hp, o_end, hipMemcpyHostToDevice, s));
      d_jobs = (Job*)d_plan;
      d_tiles = (Tile*)(d_plan + o_tiles);
      d_tile_ids = (int*)(d_plan + o_tids);
      d_job_ids = (int*)(d_plan + o_jids);
    }

    if (l == 0) {
      {
        ProfScope ps(PK_ROOT, (double)level_points, s);
        launch_root(cx, cy, cz, d_tiles, ntiles, d_jobs, njobs, f->d_trees, d_partials, (size_t)Ly.max_tiles,
                    p.reg_eps, s);
      }
      HIP_LAUNCHED();
      // a non-finite coordinate is reported after the build: the kernels stay
      // in bounds on non-finite values (such children fail their Cholesky and
      // die), so no synchronisation is spent on it here
    }

    // ---- EM for the 8 children of every job.  The block classes run on side
    // streams, concurrently with the tiled iterations on the caller's stream
    // (disjoint jobs: disjoint children, shared read-only points and plan).
    launch_init_children(d_jobs, njobs, f->d_trees, f->d_nodes, f->d_tab, p.reg_eps, s);
    bool joined[3] = {false, false, false};
    if (p.build_iters > 0 && (cls_n[0] || cls_n[1] || cls_n[2])) {
      int rc2 = ensure_side_streams(f);
      if (rc2) return rc2;
      HIP_TRY(hipEventRecord(f->ev_fork, s));
      const int nts[3] = {64, 256, 512};
      for (int c = 0; c < 3; ++c) {
        if (!cls_n[c]) continue;
        hipStream_t ss = f->side[c];
        HIP_TRY(hipStreamWaitEvent(ss, f->ev_fork, 0));
        {
          ProfScope ps(PK_EM_BLOCK, (double)cls_points[c] * p.build_iters, ss);
          launch_em_block(nts[c], cx, cy, cz, d_job_ids + cls_off[c], cls_n[c], d_jobs, f->d_tab, f->d_nodes,
                          p.build_iters, p.reg_eps, p.min_mass, ss);
        }
        HIP_TRY(hipEventRecord(f->ev_join[c], ss));
        joined[c] = true;
      }
    }
    if (nbig && p.build_iters > 0) {
      // iteration it: the E-step of every tile; the previous iteration's fold
      // and M-step either inside every tile block (few tiles: no launch in
      // between) or once per tiled job in a launch of its own
      const bool inl = nbig <= g_tune.fold_tiles;
      NodeF* chb[2] = {d_ch, (NodeF*)d_frames};
      for (int it = 0; it < p.build_iters; ++it) {
        {
          ProfScope ps(PK_EM_TILE, (double)cls_points[3], s);
          launch_em_tile(g_tune.tile_threads, cx, cy, cz, d_tiles, d_tile_ids, nbig, d_jobs, f->d_tab,
                         inl ? chb[(it + 1) & 1] : nullptr, inl ? chb[it & 1] : d_ch, inl ? nullptr : d_frames,
                         d_part[(it + 1) & 1], d_part[it & 1], (size_t)Ly.max_tiles, p.reg_eps, p.min_mass, it == 0,
                         inl, s);
        }
        if (!inl && it + 1 < p.build_iters) {
          ProfScope ps(PK_EM_MSTEP, (double)nbigjobs, s);
          launch_em_fold(d_job_ids + cls_off[3], nbigjobs, d_jobs, d_part[it & 1], (size_t)Ly.max_tiles, p.reg_eps,
                         p.min_mass, d_ch, d_frames, s);
        }
      }
      const int last = (p.build_iters - 1) & 1;
      ProfScope ps(PK_EM_MSTEP, (double)nbigjobs, s);
      launch_em_mstep(d_job_ids + cls_off[3], nbigjobs, d_jobs, f->d_tab, f->d_nodes, d_part[last],
                      (size_t)Ly.max_tiles, p.reg_eps, p.min_mass, inl ? chb[last] : d_ch, s);
    }
    for (int c = 0; c < 3; ++c)
      if (joined[c]) HIP_TRY(hipStreamWaitEvent(s, f->ev_join[c], 0));
    // ---- hard partition, child ranges, stable split, per-node statistics
    {
      ProfScope ps(PK_PARTITION, (double)level_points, s);
      launch_partition(cx, cy, cz, d_tiles, ntiles, d_jobs, f->d_tab, f->d_nodes, child, d_tile_counts, s);
    }
    launch_fill_u32(d_lvl, 0u, 2 * lvl_size[l], s);
    launch_prefix(d_jobs, njobs, d_tile_counts, d_tile_base, f->d_nodes, d_lvl, s);
    float* nx = pts[ping];
    float* ny = nx + n_total;
    float* nz = ny + n_total;
    {
      ProfScope ps(PK_SCATTER, (double)level_points, s);
      launch_scatter(cx, cy, cz, cperm, d_tiles, ntiles, d_jobs, f->d_trees, child, d_tile_base, nx, ny, nz,
                     perm[ping], f->d_labels, l, level_off(l), s);
    }
    launch_finalize_level(d_jobs, njobs, f->d_nodes, f->d_tab, s);
    HIP_LAUNCHED();
    cx = nx; cy = ny; cz = nz;
    cperm = perm[ping];
    ping ^= 1;
    if (l + 1 < Lmax) {
      HIP_TRY(hipMemcpyAsync(h_lvl, d_lvl, sizeof(int2) * lvl_size[l], hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      prof_collect();
    }
  }
  // origin, extent and status back to the host copy
  HIP_TRY(hipMemcpyAsync(h_trees + B, f->d_trees, sizeof(TreeDev) * B, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  prof_collect();
  for (int b = 0; b < B; ++b)
    if (h_trees[B + b].status != 0) return fail(HGMM_ENONFINITE, "non-finite coordinate in cloud %d", b);
  f->hint = hint;
  f->hint_key = build_shape_key(f, p);
  f->n_host_builds += 1;
  f->has_labels = true;
  return HGMM_OK;
}

// Construction with every level planned on the device (plan_level_kernel makes
// the host planner's plan) and every launch of the construction, all levels,
// in one graph whose kernels read their work counts from the level plans.
// Grids are sized from the work counts of the last host-planned construction
// of the same shape (the first call of a shape runs run_build, which records
// them); a block class or the tiled iterations of a level that had no work
// then are left out of the graph, and a call whose plan has work there is
// redone by run_build.  The graph is captured once per shape and hints
// (cloud sizes and depths, buffers, parameters, launch shapes) and cached in
// the handle; a call uploads the tree records and the per-level tree lists,
// replays the graph on the handle's stream and reads back the status and the
// level plans.  Results equal those of run_build.
static int run_build_graph(hgmm_forest_s* f, BuildInput in, const hgmm_build_params& p, char* ws, size_t ws_bytes,
                           hipStream_t s) {
  const int B = (int)f->trees.size();
  int64_t n_total = 0;
  int Lmax = 0;
  for (auto& t : f->trees) { n_total += t.n_points; Lmax = std::max(Lmax, t.levels); }
  if (f->hint_key != build_shape_key(f, p) || (int)f->hint.size() != Lmax)
    return run_build(f, in, p, ws, ws_bytes, s);
  const std::vector<std::array<int, 7>> hint = f->hint;
  BuildLayout Ly = build_layout(n_total, max_jobs_for(f->trees), max_lvl_for(f->trees), B, Lmax);
  if (ws_bytes < Ly.total) return fail(HGMM_EINVAL, "build workspace too small: %zu < %zu", ws_bytes, Ly.total);
  int rc = ensure_graph_stream(f);
  if (!rc) rc = ensure_side_streams(f);
  if (rc) return rc;
  hipStream_t gs = f->gstream;

  // per-level lists of the trees that have the level, and level-compact bases
  std::vector<std::vector<int64_t>> lvl_base(Lmax, std::vector<int64_t>(B, -1));
  std::vector<int64_t> lvl_size(Lmax, 0);
  for (int l = 0; l < Lmax; ++l)
    for (int b = 0; b < B; ++b)
      if (f->trees[b].levels > l) { lvl_base[l][b] = lvl_size[l]; lvl_size[l] += level_nodes(l); }
  std::vector<int> lt_off(Lmax + 1, 0);
  for (int l = 0; l < Lmax; ++l) {
    int c = 0;
    for (int b = 0; b < B; ++b) c += (f->trees[b].levels > l);
    lt_off[l + 1] = lt_off[l] + c;
  }
  const size_t st_trees = 0;
  const size_t st_lt = align_up(st_trees + sizeof(TreeDev) * 2 * B);
  const size_t st_plan = align_up(st_lt + sizeof(LevelTree) * (size_t)std::max(lt_off[Lmax], 1));
  const size_t st_end = align_up(st_plan + sizeof(int) * PL_SIZE * (size_t)Lmax);
  rc = grow_stage(f, st_end);
  if (rc) return rc;
  char* H = f->h_stage;
  TreeDev* h_trees = (TreeDev*)(H + st_trees);
  LevelTree* h_lt = (LevelTree*)(H + st_lt);
  int* h_plan = (int*)(H + st_plan);
  for (int b = 0; b < B; ++b) {
    TreeDev& T = h_trees[b];
    memset(&T, 0, sizeof(T));
    T.node_base = f->trees[b].node_base;
    T.point_off = f->trees[b].point_off;
    T.label_base = f->trees[b].label_base;
    T.levels = f->trees[b].levels;
    T.n_points = (int32_t)f->trees[b].n_points;
  }
  for (int l = 0; l < Lmax; ++l) {
    int c = lt_off[l];
    for (int b = 0; b < B; ++b)
      if (f->trees[b].levels > l)
        h_lt[c++] = LevelTree{b, l > 0 ? (int32_t)lvl_base[l - 1][b] : -1, (int32_t)lvl_base[l][b], 0};
  }

  float* pts[2] = {(float*)(ws + Ly.pts[0]), (float*)(ws + Ly.pts[1])};
  int* perm[2] = {(int*)(ws + Ly.perm[0]), (int*)(ws + Ly.perm[1])};
  uint8_t* child = (uint8_t*)(ws + Ly.child);
  Tile* d_tiles = (Tile*)(ws + Ly.tiles);
  int* d_tile_ids = (int*)(ws + Ly.tile_ids);
  int* d_job_ids = (int*)(ws + Ly.job_ids);
  Job* d_jobs = (Job*)(ws + Ly.jobs);
  double* d_partials = (double*)(ws + Ly.partials);
  double* d_part[2] = {d_partials, (double*)(ws + Ly.partials2)};
  // children (8 per tiled job) and the next E-step's frame (kFrameBytes per
  // tiled job) of the tiled jobs between iterations; with the fold inside
  // the tile blocks the two regions are the children's ping-pong buffers
  NodeF* d_ch = (NodeF*)(ws + Ly.chbuf);
  void* d_frames = ws + Ly.frames;
  int* d_tile_counts = (int*)(ws + Ly.tile_counts);
  int* d_tile_base = (int*)(ws + Ly.tile_base);
  int2* d_lvl = (int2*)(ws + Ly.lvl_info);
  LevelTree* d_lt = (LevelTree*)(ws + Ly.level_trees);
  int* d_plans = (int*)(ws + Ly.plans);

  uint64_t eps_bits, mm_bits;
  memcpy(&eps_bits, &p.reg_eps, 8);
  memcpy(&mm_bits, &p.min_mass, 8);
  std::vector<uint64_t> key = {(uint64_t)ws, (uint64_t)in.xs, (uint64_t)in.ys, (uint64_t)in.zs, (uint64_t)n_total,
                               (uint64_t)B, (uint64_t)Lmax, (uint64_t)f->d_trees, (uint64_t)f->d_nodes,
                               (uint64_t)f->d_tab, (uint64_t)f->d_labels, (uint64_t)p.build_iters, eps_bits, mm_bits};
  const int32_t* tv = (const int32_t*)&g_tune;
  for (size_t k = 0; k < sizeof(hgmm_tuning) / sizeof(int32_t); ++k) key.push_back((uint64_t)(uint32_t)tv[k]);
  for (auto& t : f->trees) key.push_back(((uint64_t)t.levels << 40) | (uint64_t)t.n_points);
  for (auto& h : hint)
    for (int v : h) key.push_back((uint64_t)(uint32_t)v);

  // every launch of a construction with device-planned levels, on stream gs
  // (side streams for the block classes); returns false if an event call failed
  auto enqueue = [&](hipStream_t gs) -> bool {
    // grids from the hinted work counts with some slack; the kernels loop
    // over their work items, so any count is covered
    const int mj = (int)Ly.max_jobs, mt = (int)Ly.max_tiles;
    auto grid = [](int h, int cap) { return std::max(1, std::min(cap, h + h / 8 + 8)); };
    const int nts[3] = {64, 256, 512};
    const int64_t nodes_total = f->total_nodes();
    launch_fill_u32(f->d_nodes, 0u, (int64_t)(sizeof(NodeD) / 4) * nodes_total, gs);
    launch_fill_u32(f->d_tab, 0u, (int64_t)(sizeof(NodeF) / 4) * nodes_total, gs);
    int64_t nlab = 0;
    for (auto& t : f->trees) nlab += (int64_t)t.levels * t.n_points;
    launch_fill_u32(f->d_labels, 0xFFFFFFFFu, nlab, gs);
    const float* cx = in.xs;
    const float* cy = in.ys;
    const float* cz = in.zs;
    const int* cperm = nullptr;
    int ping = 0;
    bool ok = true;
    for (int l = 0; l < Lmax && ok; ++l) {
      const int* pl = d_plans + (size_t)l * PL_SIZE;
      const std::array<int, 7>& h = hint[l];
      const int G_jobs = grid(h[0], mj), G_tiles = grid(h[1], mt), G_tile = grid(h[2], mt), G_mstep = grid(h[6], mj);
      const int G_thr = G_jobs;
      const int G_block[3] = {grid(h[3], mj), grid(h[4], mj), grid(h[5], mj)};
      launch_plan_level(d_lt + lt_off[l], lt_off[l + 1] - lt_off[l], l == 0 ? 1 : (int)level_nodes(l - 1), l,
                        l > 0 ? level_off(l - 1) : 0, level_off(l), d_lvl, f->d_trees, g_tune.block64_max,
                        g_tune.block256_max, g_tune.block512_max, g_tune.target_tiles, g_tune.min_tile,
                        g_tune.max_tile, mj, mt, d_jobs, d_job_ids, d_tiles, d_tile_ids, (int*)pl, gs);
      if (l == 0)
        launch_root(cx, cy, cz, d_tiles, G_tiles, d_jobs, G_jobs, f->d_trees, d_partials, (size_t)Ly.max_tiles,
                    p.reg_eps, gs, pl + PL_NTILES, pl + PL_NJOBS);
      launch_init_children(d_jobs, G_thr, f->d_trees, f->d_nodes, f->d_tab, p.reg_eps, gs, pl + PL_NJOBS);
      if (p.build_iters > 0) {
        ok = ok && hipEventRecord(f->ev_fork, gs) == hipSuccess;
        for (int c = 0; c < 3 && ok; ++c) {
          if (h[3 + c] == 0) continue;  // no job of this class in the hinted plan
          ok = ok && hipStreamWaitEvent(f->side[c], f->ev_fork, 0) == hipSuccess;
          launch_em_block(nts[c], cx, cy, cz, d_job_ids, G_block[c], d_jobs, f->d_tab, f->d_nodes, p.build_iters,
                          p.reg_eps, p.min_mass, f->side[c], pl + PL_CLS_N + c, pl + PL_CLS_OFF + c);
          ok = ok && hipEventRecord(f->ev_join[c], f->side[c]) == hipSuccess;
        }
        if (h[2] > 0) {  // tiled parents in the hinted plan
          const bool inl = h[2] <= g_tune.fold_tiles;
          NodeF* chb[2] = {d_ch, (NodeF*)d_frames};
          for (int it = 0; it < p.build_iters; ++it) {
            launch_em_tile(g_tune.tile_threads, cx, cy, cz, d_tiles, d_tile_ids, G_tile, d_jobs, f->d_tab,
                           inl ? chb[(it + 1) & 1] : nullptr, inl ? chb[it & 1] : d_ch, inl ? nullptr : d_frames,
                           d_part[(it + 1) & 1], d_part[it & 1], (size_t)Ly.max_tiles, p.reg_eps, p.min_mass,
                           it == 0, inl, gs, pl + PL_NBIG);
            if (!inl && it + 1 < p.build_iters)
              launch_em_fold(d_job_ids, G_mstep, d_jobs, d_part[it & 1], (size_t)Ly.max_tiles, p.reg_eps, p.min_mass,
                             d_ch, d_frames, gs, pl + PL_CLS_N + 3, pl + PL_CLS_OFF + 3);
          }
          const int last = (p.build_iters - 1) & 1;
          launch_em_mstep(d_job_ids, G_mstep, d_jobs, f->d_tab, f->d_nodes, d_part[last], (size_t)Ly.max_tiles,
                          p.reg_eps, p.min_mass, inl ? chb[last] : d_ch, gs, pl + PL_CLS_N + 3, pl + PL_CLS_OFF + 3);
        }
        for (int c = 0; c < 3 && ok; ++c)
          if (h[3 + c] > 0) ok = ok && hipStreamWaitEvent(gs, f->ev_join[c], 0) == hipSuccess;
      }
      launch_partition(cx, cy, cz, d_tiles, G_tiles, d_jobs, f->d_tab, f->d_nodes, child, d_tile_counts, gs,
                       pl + PL_NTILES);
      launch_fill_u32(d_lvl, 0u, 2 * lvl_size[l], gs);
      launch_prefix(d_jobs, G_jobs, d_tile_counts, d_tile_base, f->d_nodes, d_lvl, gs, pl + PL_NJOBS);
      float* nx = pts[ping];
      float* ny = nx + n_total;
      float* nz = ny + n_total;
      launch_scatter(cx, cy, cz, cperm, d_tiles, G_tiles, d_jobs, f->d_trees, child, d_tile_base, nx, ny, nz,
                     perm[ping], f->d_labels, l, level_off(l), gs, pl + PL_NTILES);
      launch_finalize_level(d_jobs, G_thr, f->d_nodes, f->d_tab, gs, pl + PL_NJOBS);
      cx = nx; cy = ny; cz = nz;
      cperm = perm[ping];
      ping ^= 1;
    }
    return ok;
  };
  const bool stream_mode = g_tune.build_graph == 2;
  if (stream_mode) {
    // the same launches without a graph: the inputs, then the launches on the
    // handle's stream, with no host round trip between levels
    HIP_TRY(hipMemcpyAsync(f->d_trees, h_trees, sizeof(TreeDev) * B, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_lt, h_lt, sizeof(LevelTree) * (size_t)std::max(lt_off[Lmax], 1), hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipEventRecord(f->ev_g0, s));
    HIP_TRY(hipStreamWaitEvent(gs, f->ev_g0, 0));
    if (!enqueue(gs)) return fail(HGMM_EHIP, "construction launch sequence failed");
    HIP_LAUNCHED();
  } else if (!f->bld_exec || f->bld_key != key) {
    if (f->bld_exec) { (void)hipGraphExecDestroy(f->bld_exec); f->bld_exec = nullptr; }
    f->bld_key.clear();
    HIP_TRY(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    const bool ok = enqueue(gs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(gs, &graph);
    if (!ok || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(HGMM_EHIP, "construction graph capture failed: %s", hipGetErrorString(ec));
    }
    const hipError_t ei = hipGraphInstantiate(&f->bld_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) { f->bld_exec = nullptr; return fail(HGMM_EHIP, "construction graph instantiation failed"); }
    f->bld_key = key;
    f->n_graph_captures += 1;
  }
  if (!stream_mode) {
    // inputs of this call, then the graph on the handle's stream
    HIP_TRY(hipMemcpyAsync(f->d_trees, h_trees, sizeof(TreeDev) * B, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_lt, h_lt, sizeof(LevelTree) * (size_t)std::max(lt_off[Lmax], 1), hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipEventRecord(f->ev_g0, s));
    HIP_TRY(hipStreamWaitEvent(gs, f->ev_g0, 0));
    HIP_TRY(hipGraphLaunch(f->bld_exec, gs));
  }
  HIP_TRY(hipEventRecord(f->ev_g1, gs));
  HIP_TRY(hipStreamWaitEvent(s, f->ev_g1, 0));
  // origin, extent and status, and the plans' overflow flags
  HIP_TRY(hipMemcpyAsync(h_trees + B, f->d_trees, sizeof(TreeDev) * B, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(h_plan, d_plans, sizeof(int) * PL_SIZE * Lmax, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int l = 0; l < Lmax; ++l)
    if (h_plan[l * PL_SIZE + PL_ERR]) return fail(HGMM_EINVAL, "internal: device plan overflow at level %d", l);
  // work in a phase the graph leaves out: redo the construction host-planned
  for (int l = 0; l < Lmax; ++l) {
    const int* pl = h_plan + l * PL_SIZE;
    bool missed = hint[l][2] == 0 && p.build_iters > 0 && pl[PL_NBIG] > 0;
    for (int c = 0; c < 3; ++c) missed = missed || (hint[l][3 + c] == 0 && p.build_iters > 0 && pl[PL_CLS_N + c] > 0);
    if (missed) return run_build(f, in, p, ws, ws_bytes, s);
  }
  f->n_graph_replays += 1;  // device-planned: a graph replay, or the same launches on the stream
  for (int b = 0; b < B; ++b)
    if (h_trees[B + b].status != 0) return fail(HGMM_ENONFINITE, "non-finite coordinate in cloud %d", b);
  f->has_labels = true;
  return HGMM_OK;
}

// ---------------------------------------------------------------------------
// registration
// ---------------------------------------------------------------------------

struct RegRun {
  int max_iters;
  double lambda_c, tol_rot, tol_trans_rel;
  int max_levels;  // 0: every level of the tree
  int flat_level = -1;  // >= 0: single-level E-step over this level instead of the descent
  double soft_tau = 0.0;  // > 0: soft multi-path E-step with this pruning threshold instead of the descent
  // host staging supplied by the caller (nullptr: the handle's pinned
  // staging, grown on demand); set, the run also takes neither the graph path
  // nor the profiling events, so it allocates nothing
  char* stage = nullptr;
  size_t stage_bytes = 0;
  // with reg_sort: the Morton order of the moving points is already in the
  // workspace, left by an earlier run over the same points, forest and
  // workspace (the keys depend on the points and the trees' frames, not on
  // the poses), so the sort is skipped
  bool sorted = false;
};

static int run_register(hgmm_forest_s* f, const float* xs, const float* ys, const float* zs,
                        const std::vector<int64_t>& offs, const double* R0, const double* t0, int per_pair,
                        const RegRun& rr, char* ws, size_t ws_bytes, hipStream_t s, int mode_estep,
                        int32_t* stop_out, float* gamma_out, double* bins_ext, PoseState* h_out, double* h_norm,
                        const int32_t* active = nullptr) {
  const int P = (int)offs.size() - 1;
  const int64_t n_total = offs.back();
  const int64_t nodes_total = f->total_nodes();
  RegLayout Ly = reg_layout(n_total, nodes_total, P);
  if (ws_bytes < Ly.total) return fail(HGMM_EINVAL, "register workspace too small: %zu < %zu", ws_bytes, Ly.total);
  double* d_bins = bins_ext ? bins_ext : (double*)(ws + Ly.bins);
  PoseState* d_state = (PoseState*)(ws + Ly.state);
  int64_t* d_nmov = (int64_t*)(ws + Ly.nmov);
  Tile* d_tiles = (Tile*)(ws + Ly.tiles);
  double* d_out = (double*)(ws + Ly.out);
  double* d_pose0 = (double*)(ws + Ly.pose);
  FixBin* d_fbins = (FixBin*)(ws + Ly.fbins);
  NodeR* d_regf = (NodeR*)(ws + Ly.regf);
  int2* d_ptiles = (int2*)(ws + Ly.ptiles);

  // staging: tiles | per-pair inputs (the device layout from Ly.ptiles on) |
  // results | normal-equation sums
  size_t s_tiles = 0;
  size_t s_up = align_up(s_tiles + sizeof(Tile) * Ly.max_tiles);
  size_t s_pt = s_up;
  size_t s_nmov = s_up + (Ly.nmov - Ly.ptiles);
  size_t s_pose = s_up + (Ly.pose - Ly.ptiles);
  size_t s_act = s_up + (Ly.active - Ly.ptiles);
  size_t s_res = align_up(s_act + sizeof(int) * P);
  size_t s_norm = align_up(s_res + sizeof(PoseState) * P);
  size_t s_end = align_up(s_norm + sizeof(double) * 28 * P);
  const bool fixed_stage = rr.stage != nullptr;
  char* H = rr.stage;
  if (fixed_stage) {
    if (s_end > rr.stage_bytes)
      return fail(HGMM_EINVAL, "host staging of %zu bytes needed, %zu available", s_end, rr.stage_bytes);
  } else {
    int rc = grow_stage(f, s_end);
    if (rc) return rc;
    H = f->h_stage;
  }
  Tile* h_tiles = (Tile*)(H + s_tiles);
  int64_t* h_nmov = (int64_t*)(H + s_nmov);
  double* h_pose = (double*)(H + s_pose);
  PoseState* h_res = (PoseState*)(H + s_res);
  double* h_nrm = (double*)(H + s_norm);
  int2* h_pt = (int2*)(H + s_pt);
  int* h_act = (int*)(H + s_act);
  int* d_act = (int*)(ws + Ly.active);

  int ntiles = 0;
  const int rt = g_tune.reg_tile;
  for (int b = 0; b < P; ++b) {
    h_nmov[b] = offs[b + 1] - offs[b];
    h_pt[b].x = ntiles;
    for (int64_t st0 = offs[b]; st0 < offs[b + 1]; st0 += rt) {
      Tile& T = h_tiles[ntiles++];
      T.start = (int32_t)st0;
      T.end = (int32_t)std::min<int64_t>(offs[b + 1], st0 + rt);
      T.job = b;
      T.pad = 0;
    }
    h_pt[b].y = ntiles - h_pt[b].x;
  }
  if (ntiles > Ly.max_tiles) return fail(HGMM_EINVAL, "internal: registration tile overflow");
  const int npose = per_pair ? P : 1;
  for (int b = 0; b < npose; ++b) {
    for (int i = 0; i < 9; ++i) h_pose[12 * b + i] = R0 ? R0[9 * b + i] : (i % 4 == 0 ? 1.0 : 0.0);
    for (int i = 0; i < 3; ++i) h_pose[12 * b + 9 + i] = t0 ? t0[3 * b + i] : 0.0;
  }
  if (active)
    for (int b = 0; b < P; ++b) h_act[b] = active[b] ? 1 : 0;
  // two uploads: the tiles, then the per-pair block (up to the active flags
  // when given, else up to the start poses in use; pose rows are 12 doubles)
  HIP_TRY(hipMemcpyAsync(d_tiles, h_tiles, sizeof(Tile) * ntiles, hipMemcpyHostToDevice, s));
  const size_t up_bytes = active ? (Ly.active - Ly.ptiles) + sizeof(int) * P
                                 : (Ly.pose - Ly.ptiles) + sizeof(double) * 12 * npose;
  HIP_TRY(hipMemcpyAsync(d_ptiles, h_pt, up_bytes, hipMemcpyHostToDevice, s));
  const int* d_perm = nullptr;
  if (g_tune.reg_sort && n_total > 0) {
    float* sx = (float*)(ws + Ly.sxyz);
    float* sy = sx + n_total;
    float* sz = sy + n_total;
    if (!rr.sorted)
      HIP_TRY(launch_sort_points(xs, ys, zs, d_tiles, ntiles, f->d_trees, P, n_total, (uint64_t*)(ws + Ly.keys),
                                 (uint64_t*)(ws + Ly.keys2), (int*)(ws + Ly.vals), (int*)(ws + Ly.perm),
                                 ws + Ly.sort_temp, Ly.sort_temp_bytes, sx, sy, sz, s));
    xs = sx; ys = sy; zs = sz;
    d_perm = (const int*)(ws + Ly.perm);
  }
  launch_fill_u32(d_bins, 0u, 2 * 6 * nodes_total, s);
  launch_fill_u32(d_fbins, 0u, (int64_t)(sizeof(FixBin) / 4) * nodes_total, s);
  launch_set_stop_flags(f->d_tab, f->d_nodes, nodes_total, rr.lambda_c, s);
  launch_reg_table(f->d_tab, f->d_nodes, d_regf, nodes_total, rr.lambda_c, s);
  launch_init_pose(d_state, P, d_pose0, d_pose0 + 9, per_pair ? 12 : 0, active ? d_act : nullptr, s);
  HIP_LAUNCHED();
  const bool flat = rr.flat_level >= 0;
  const bool soft = rr.soft_tau > 0.0;
  // the descent's moments as FP64 atomic adds (compared against the
  // fixed-point default)
  const bool fp64_atomics = g_tune.reg_atomics != 0 && !flat && !soft;
  int max_tree_levels = 1;
  for (auto& tr : f->trees) max_tree_levels = std::max(max_tree_levels, tr.levels);
  // one E-step launch (descent, or the single-level scan) and one M-step launch
  NodeR* d_flatf = (NodeR*)(ws + Ly.flatf);
  if (flat) launch_flat_table(f->d_tab, f->d_nodes, d_flatf, nodes_total, s);
  auto estep = [&](hipStream_t q, int32_t* so, float* go, const int* pm, unsigned long long* wk) {
    if (soft)
      launch_soft_estep(xs, ys, zs, d_tiles, ntiles, rt, max_tree_levels, f->d_trees, f->d_tab, f->d_nodes, d_state,
                        d_bins,
                        (float)rr.soft_tau, so, pm, q);
    else if (flat)
      launch_flat_estep(xs, ys, zs, d_tiles, ntiles, rt, f->d_trees, d_flatf, d_state, d_bins, so, go, pm,
                        rr.flat_level, q);
    else
      launch_descend(xs, ys, zs, d_tiles, ntiles, f->d_trees, d_regf, d_state, d_fbins,
                     fp64_atomics ? d_bins : nullptr, so, go, pm, g_tune.reg_lds_levels, rr.max_levels, wk, q);
  };
  auto mstep = [&](hipStream_t q) {
    launch_normal(d_bins, d_fbins, f->d_nodes, f->d_trees, d_state, d_nmov, P, (flat || soft || fp64_atomics) ? 2 : 0,
                  rr.tol_rot, rr.tol_trans_rel, rr.max_iters, d_out, q);
  };
  if (mode_estep) {
    estep(s, stop_out, gamma_out, d_perm, nullptr);
    if (!flat && !soft && !fp64_atomics) launch_fold_bins(f->d_trees, d_fbins, d_bins, P, s);
    if (h_norm) {
      launch_normal(d_bins, d_fbins, f->d_nodes, f->d_trees, d_state, d_nmov, P, 1, 0.0, 0.0, 1,
                    d_out, s);
      HIP_TRY(hipMemcpyAsync(h_nrm, d_out, sizeof(double) * 28 * P, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      memcpy(h_norm, h_nrm, sizeof(double) * 28 * P);
    }
    HIP_LAUNCHED();
    return HGMM_OK;
  }
  // E/M iterations in chunks; between chunks the host checks whether every
  // pair has converged so that no further launches are queued
  int it = 0;
  const int chunk = std::max(1, g_tune.reg_chunk);
  if (g_tune.reg_graph && !g_prof.on && !fixed_stage) {
    int rc2 = ensure_graph_stream(f);
    if (rc2) return rc2;
    uint64_t tr, tt, soft_key;
    memcpy(&soft_key, &rr.soft_tau, 8);
    memcpy(&tr, &rr.tol_rot, 8);
    memcpy(&tt, &rr.tol_trans_rel, 8);
    const std::vector<uint64_t> key = {(uint64_t)xs, (uint64_t)ys, (uint64_t)zs, (uint64_t)d_tiles, (uint64_t)ntiles,
                                       (uint64_t)f->d_trees, (uint64_t)f->d_tab, (uint64_t)f->d_nodes,
                                       (uint64_t)d_state, (uint64_t)d_bins, (uint64_t)d_fbins,
                                       (uint64_t)g_tune.reg_tile, (uint64_t)g_tune.reg_lds_levels,
                                       (uint64_t)g_tune.reg_atomics,
                                       (uint64_t)d_ptiles, (uint64_t)d_nmov, (uint64_t)P, (uint64_t)chunk, tr, tt,
                                       (uint64_t)rr.max_iters, (uint64_t)rr.max_levels, (uint64_t)d_out,
                                       (uint64_t)(int64_t)rr.flat_level, soft_key};
    if (!f->reg_exec || f->reg_key != key) {
      if (f->reg_exec) { (void)hipGraphExecDestroy(f->reg_exec); f->reg_exec = nullptr; }
      f->reg_key.clear();
      HIP_TRY(hipStreamBeginCapture(f->gstream, hipStreamCaptureModeThreadLocal));
      for (int c = 0; c < chunk; ++c) {
        estep(f->gstream, nullptr, nullptr, nullptr, nullptr);
        mstep(f->gstream);
      }
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(f->gstream, &graph);
      if (ec != hipSuccess || !graph) return fail(HGMM_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&f->reg_exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) { f->reg_exec = nullptr; return fail(HGMM_EHIP, "graph instantiation failed"); }
      f->reg_key = key;
    }
    HIP_TRY(hipEventRecord(f->ev_g0, s));
    HIP_TRY(hipStreamWaitEvent(f->gstream, f->ev_g0, 0));
    while (it < rr.max_iters) {
      HIP_TRY(hipGraphLaunch(f->reg_exec, f->gstream));
      it += chunk;
      HIP_TRY(hipMemcpyAsync(h_res, d_state, sizeof(PoseState) * P, hipMemcpyDeviceToHost, f->gstream));
      HIP_TRY(hipStreamSynchronize(f->gstream));
      bool all_done = true;
      for (int b = 0; b < P; ++b) all_done = all_done && (h_res[b].done != 0);
      if (all_done) break;
    }
    HIP_TRY(hipEventRecord(f->ev_g1, f->gstream));
    HIP_TRY(hipStreamWaitEvent(s, f->ev_g1, 0));
    memcpy(h_out, h_res, sizeof(PoseState) * P);
    return HGMM_OK;
  }
  while (it < rr.max_iters) {
    const int end = std::min(rr.max_iters, it + chunk);
    for (; it < end; ++it) {
      {
        ProfScope ps(soft ? PK_SOFT : flat ? PK_FLAT : PK_DESCEND, (double)n_total, s, it, !fixed_stage);
        estep(s, nullptr, nullptr, nullptr, (!soft && !flat) ? ps.work_slot() : nullptr);
      }
      {
        ProfScope ps(PK_NORMAL, (double)nodes_total, s, it, !fixed_stage);
        mstep(s);
      }
    }
    HIP_LAUNCHED();
    HIP_TRY(hipMemcpyAsync(h_res, d_state, sizeof(PoseState) * P, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool all_done = true;
    for (int b = 0; b < P; ++b) all_done = all_done && (h_res[b].done != 0);
    if (all_done) break;
  }
  {
    int done_iters = 0;
    for (int b = 0; b < P; ++b) done_iters = std::max(done_iters, (int)h_res[b].iters);
    prof_collect(done_iters);
  }
  memcpy(h_out, h_res, sizeof(PoseState) * P);
  return HGMM_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* hgmm_last_error(void) { return g_err.c_str(); }

int hgmm_params_default(hgmm_build_params* bp, hgmm_reg_params* rp) {
  if (bp) { bp->levels = 2; bp->build_iters = 30; bp->reg_eps = 1e-6; bp->min_mass = 1.0; }
  if (rp) { rp->max_iters = 30; rp->max_levels = 0; rp->lambda_c = 0.01; rp->tol_rot = 1e-6; rp->tol_trans_rel = 1e-6; }
  return HGMM_OK;
}

int64_t hgmm_tree_nodes(int levels) {
  if (levels < 1 || levels > HGMM_MAX_LEVELS) return -1;
  return tree_nodes(levels);
}

int hgmm_build_graph_stats(hgmm_tree tree, int64_t* replays, int64_t* captures, int64_t* host_builds) {
  if (!tree || !replays || !captures || !host_builds) return fail(HGMM_EINVAL, "null pointer argument");
  *replays = tree->n_graph_replays;
  *captures = tree->n_graph_captures;
  *host_builds = tree->n_host_builds;
  return HGMM_OK;
}

int64_t hgmm_level_offset(int level) {
  if (level < 0 || level > HGMM_MAX_LEVELS) return -1;
  return level_off(level);
}

size_t hgmm_build_workspace_bytes(int64_t n, int levels) {
  if (levels < 1 || levels > HGMM_MAX_LEVELS || n < 0) return 0;
  std::vector<TreeHost> t(1);
  t[0].levels = levels;
  t[0].n_points = n;
  return build_layout(n, max_jobs_for(t), max_lvl_for(t), 1, levels).total;
}

size_t hgmm_register_workspace_bytes(int64_t n, int levels) {
  if (levels < 1 || levels > HGMM_MAX_LEVELS || n < 0) return 0;
  return reg_layout(n, tree_nodes(levels), 1).total;
}

static int check_build_params(const hgmm_build_params* p) {
  if (!p) return fail(HGMM_EINVAL, "null build params");
  if (p->levels < 1 || p->levels > HGMM_MAX_LEVELS) return fail(HGMM_EINVAL, "levels %d outside [1, 6]", p->levels);
  if (p->build_iters < 0) return fail(HGMM_EINVAL, "build_iters < 0");
  if (!(p->reg_eps > 0.0) || !std::isfinite(p->reg_eps)) return fail(HGMM_EINVAL, "reg_eps must be positive");
  if (!(p->min_mass >= 0.0)) return fail(HGMM_EINVAL, "min_mass must be >= 0");
  return HGMM_OK;
}

int hgmm_build(const float* d_xyz, int64_t n, const hgmm_build_params* p, void* d_ws, size_t ws_bytes, void* stream,
               hgmm_tree* tree) {
  int rc = check_build_params(p);
  if (rc) return rc;
  if (!d_xyz || !d_ws || !tree) return fail(HGMM_EINVAL, "null pointer argument");
  if (n < 8) return fail(HGMM_ETOOFEW, "need at least 8 points, got %lld", (long long)n);
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  hgmm_forest_s* f = *tree;
  const bool fresh = (f == nullptr);
  if (fresh) f = new hgmm_forest_s();
  HIP_TRY(hipGetDevice(&f->device));
  f->trees.assign(1, TreeHost{p->levels, n, 0, 0, 0});
  rc = setup_forest(f);
  if (!rc) {
    BuildInput in{d_xyz, d_xyz + n, d_xyz + 2 * n};
    rc = (g_tune.build_graph && !g_prof.on) ? run_build_graph(f, in, *p, (char*)d_ws, ws_bytes, (hipStream_t)stream)
                                            : run_build(f, in, *p, (char*)d_ws, ws_bytes, (hipStream_t)stream);
  }
  if (rc && fresh) { free_forest(f); return rc; }
  *tree = f;
  return rc;
}

int hgmm_register(hgmm_tree tree, const float* d_xyz, int64_t n, const hgmm_reg_params* p, const double* R0,
                  const double* t0, void* d_ws, size_t ws_bytes, void* stream, double R[9], double t[3], int* iters,
                  double* loglik) {
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (!tree || !d_xyz || !p || !d_ws || !R || !t || !iters) return fail(HGMM_EINVAL, "null pointer argument");
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  if (p->max_iters < 1) return fail(HGMM_EINVAL, "max_iters must be >= 1");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_register takes a single-tree handle");
  std::vector<int64_t> offs = {0, n};
  RegRun rr{p->max_iters, p->lambda_c, p->tol_rot, p->tol_trans_rel, p->max_levels};
  PoseState res;
  int rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R0, t0, 0, rr, (char*)d_ws, ws_bytes,
                        (hipStream_t)stream, 0, nullptr, nullptr, nullptr, &res, nullptr);
  if (rc) return rc;
  for (int i = 0; i < 9; ++i) R[i] = res.R[i];
  for (int i = 0; i < 3; ++i) t[i] = res.t[i];
  *iters = res.iters;
  if (loglik) *loglik = res.loglik;
  if (res.status != 0) return fail(res.status, "normal equations not positive definite at iteration %d", res.iters);
  return HGMM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free registration: the workspace lives in a static device array
// ---------------------------------------------------------------------------
//
// Callers that may not allocate (code under stream capture, serving loops)
// register against a static device array instead of a caller workspace.  In
// host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress and
// only that address is ever handed to kernels or copies.  Every call on a
// device shares that device's array (and the process-wide host staging), so
// calls that overlap in time race; the array keeps the last call's contents,
// and the registration clears what it accumulates into before use.

static __device__ __align__(256) char scratch[HGMM_NOALLOC_SCRATCH_BYTES];
constexpr size_t kNoAllocStageBytes = size_t(1) << 18;
alignas(256) static char g_noalloc_stage[kNoAllocStageBytes];
static void* g_scratch_ptr[HGMM_NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of this device's scratch, looked up on the first call on
// the device with that device current.
static int noalloc_scratch(char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= HGMM_NOALLOC_MAX_DEVICES) return fail(HGMM_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HGMM_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return HGMM_OK;
}

extern "C" {

size_t hgmm_noalloc_scratch_bytes(void) { return HGMM_NOALLOC_SCRATCH_BYTES; }

int hgmm_register_noalloc(hgmm_tree tree, const float* d_xyz, int64_t n, const hgmm_reg_params* p, const double* R0,
                          const double* t0, void* stream, double R[9], double t[3], int* iters, double* loglik) {
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (!tree || !d_xyz || !p || !R || !t || !iters) return fail(HGMM_EINVAL, "null pointer argument");
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  if (p->max_iters < 1) return fail(HGMM_EINVAL, "max_iters must be >= 1");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_register_noalloc takes a single-tree handle");
  const size_t need = reg_layout(n, tree->total_nodes(), 1).total;
  if (need > HGMM_NOALLOC_SCRATCH_BYTES)
    return fail(HGMM_EINVAL, "%lld points on a %lld-node tree need %zu bytes of scratch; the static scratch holds %zu",
                (long long)n, (long long)tree->total_nodes(), need, (size_t)HGMM_NOALLOC_SCRATCH_BYTES);
  char* ws = nullptr;
  int rc = noalloc_scratch(&ws);
  if (rc) return rc;
  std::vector<int64_t> offs = {0, n};
  RegRun rr{p->max_iters, p->lambda_c, p->tol_rot, p->tol_trans_rel, p->max_levels};
  rr.stage = g_noalloc_stage;
  rr.stage_bytes = kNoAllocStageBytes;
  PoseState res;
  rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R0, t0, 0, rr, ws, need, (hipStream_t)stream, 0,
                    nullptr, nullptr, nullptr, &res, nullptr);
  if (rc) return rc;
  for (int i = 0; i < 9; ++i) R[i] = res.R[i];
  for (int i = 0; i < 3; ++i) t[i] = res.t[i];
  *iters = res.iters;
  if (loglik) *loglik = res.loglik;
  if (res.status != 0) return fail(res.status, "normal equations not positive definite at iteration %d", res.iters);
  return HGMM_OK;
}

int hgmm_estep(hgmm_tree tree, const float* d_xyz, int64_t n, const double R[9], const double t[3], double lambda_c,
               void* d_ws, size_t ws_bytes, void* stream, int32_t* d_stop_node, float* d_gamma, double* d_bins,
               double* loglik) {
  if (!tree || !d_xyz || !R || !t || !d_ws) return fail(HGMM_EINVAL, "null pointer argument");
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_estep takes a single-tree handle");
  std::vector<int64_t> offs = {0, n};
  RegRun rr{1, lambda_c, 0.0, 0.0, 0};
  double nrm[28];
  int rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R, t, 0, rr, (char*)d_ws, ws_bytes,
                        (hipStream_t)stream, 1, d_stop_node, d_gamma, d_bins, nullptr, loglik ? nrm : nullptr);
  if (rc) return rc;
  if (loglik) *loglik = nrm[27];
  return HGMM_OK;
}

static int check_flat_level(hgmm_tree tree, int level) {
  int lmin = 1 << 30;
  for (auto& t : tree->trees) lmin = std::min(lmin, t.levels);
  if (level < 0 || level >= lmin)
    return fail(HGMM_EINVAL, "level %d outside the tree's levels 0..%d", level, lmin - 1);
  return HGMM_OK;
}

int hgmm_register_flat(hgmm_tree tree, const float* d_xyz, int64_t n, int level, const hgmm_reg_params* p,
                       const double* R0, const double* t0, void* d_ws, size_t ws_bytes, void* stream, double R[9],
                       double t[3], int* iters, double* loglik) {
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (!tree || !d_xyz || !p || !d_ws || !R || !t || !iters) return fail(HGMM_EINVAL, "null pointer argument");
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  if (p->max_iters < 1) return fail(HGMM_EINVAL, "max_iters must be >= 1");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_register_flat takes a single-tree handle");
  int rc = check_flat_level(tree, level);
  if (rc) return rc;
  std::vector<int64_t> offs = {0, n};
  RegRun rr{p->max_iters, 0.0, p->tol_rot, p->tol_trans_rel, 0, level};
  PoseState res;
  rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R0, t0, 0, rr, (char*)d_ws, ws_bytes,
                    (hipStream_t)stream, 0, nullptr, nullptr, nullptr, &res, nullptr);
  if (rc) return rc;
  for (int i = 0; i < 9; ++i) R[i] = res.R[i];
  for (int i = 0; i < 3; ++i) t[i] = res.t[i];
  *iters = res.iters;
  if (loglik) *loglik = res.loglik;
  if (res.status != 0) return fail(res.status, "normal equations not positive definite at iteration %d", res.iters);
  return HGMM_OK;
}

int hgmm_estep_flat(hgmm_tree tree, const float* d_xyz, int64_t n, int level, const double R[9], const double t[3],
                    void* d_ws, size_t ws_bytes, void* stream, int32_t* d_stop_node, float* d_gamma, double* d_bins,
                    double* loglik) {
  if (!tree || !d_xyz || !R || !t || !d_ws) return fail(HGMM_EINVAL, "null pointer argument");
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_estep_flat takes a single-tree handle");
  int rc = check_flat_level(tree, level);
  if (rc) return rc;
  std::vector<int64_t> offs = {0, n};
  RegRun rr{1, 0.0, 0.0, 0.0, 0, level};
  double nrm[28];
  rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R, t, 0, rr, (char*)d_ws, ws_bytes,
                    (hipStream_t)stream, 1, d_stop_node, d_gamma, d_bins, nullptr, loglik ? nrm : nullptr);
  if (rc) return rc;
  if (loglik) *loglik = nrm[27];
  return HGMM_OK;
}

int hgmm_point_loglik(hgmm_tree tree, const float* d_xyz, int64_t n, const double R[9], const double t[3],
                      double lambda_c, void* d_ws, size_t ws_bytes, void* stream, int32_t* d_node, float* d_loglik) {
  if (!tree || !d_xyz || !R || !t || !d_ws || !d_loglik) return fail(HGMM_EINVAL, "null pointer argument");
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_point_loglik takes a single-tree handle");
  const RegLayout Ly = reg_layout(n, tree->total_nodes(), 1);
  if (ws_bytes < Ly.total) return fail(HGMM_EINVAL, "workspace too small: %zu < %zu", ws_bytes, Ly.total);
  // stop nodes in the caller's buffer, else in the sort's value scratch (free
  // once the points are ordered)
  int32_t* stop = d_node ? d_node : (int32_t*)((char*)d_ws + Ly.vals);
  std::vector<int64_t> offs = {0, n};
  RegRun rr{1, lambda_c, 0.0, 0.0, 0};
  int rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R, t, 0, rr, (char*)d_ws, ws_bytes,
                        (hipStream_t)stream, 1, stop, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  launch_point_loglik(d_xyz, d_xyz + n, d_xyz + 2 * n, n, stop, tree->d_trees, tree->d_nodes,
                      (const PoseState*)((char*)d_ws + Ly.state), d_loglik, (hipStream_t)stream);
  HIP_LAUNCHED();
  return HGMM_OK;
}

static int check_tau(double tau) {
  if (!(tau > 0.0 && tau < 1.0)) return fail(HGMM_EINVAL, "pruning threshold tau must be in (0, 1)");
  return HGMM_OK;
}

int hgmm_register_soft(hgmm_tree tree, const float* d_xyz, int64_t n, double tau, const hgmm_reg_params* p,
                       const double* R0, const double* t0, void* d_ws, size_t ws_bytes, void* stream, double R[9],
                       double t[3], int* iters, double* loglik) {
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (!tree || !d_xyz || !p || !d_ws || !R || !t || !iters) return fail(HGMM_EINVAL, "null pointer argument");
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  if (p->max_iters < 1) return fail(HGMM_EINVAL, "max_iters must be >= 1");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_register_soft takes a single-tree handle");
  int rc = check_tau(tau);
  if (rc) return rc;
  std::vector<int64_t> offs = {0, n};
  RegRun rr{p->max_iters, p->lambda_c, p->tol_rot, p->tol_trans_rel, 0, -1, tau};
  PoseState res;
  rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R0, t0, 0, rr, (char*)d_ws, ws_bytes,
                    (hipStream_t)stream, 0, nullptr, nullptr, nullptr, &res, nullptr);
  if (rc) return rc;
  for (int i = 0; i < 9; ++i) R[i] = res.R[i];
  for (int i = 0; i < 3; ++i) t[i] = res.t[i];
  *iters = res.iters;
  if (loglik) *loglik = res.loglik;
  if (res.status != 0) return fail(res.status, "normal equations not positive definite at iteration %d", res.iters);
  return HGMM_OK;
}

int hgmm_estep_soft(hgmm_tree tree, const float* d_xyz, int64_t n, double tau, const double R[9], const double t[3],
                    double lambda_c, void* d_ws, size_t ws_bytes, void* stream, int32_t* d_stops, double* d_bins,
                    double* loglik) {
  if (!tree || !d_xyz || !R || !t || !d_ws) return fail(HGMM_EINVAL, "null pointer argument");
  if (n < 1) return fail(HGMM_ETOOFEW, "empty cloud");
  if (n > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "hgmm_estep_soft takes a single-tree handle");
  int rc = check_tau(tau);
  if (rc) return rc;
  std::vector<int64_t> offs = {0, n};
  RegRun rr{1, lambda_c, 0.0, 0.0, 0, -1, tau};
  double nrm[28];
  rc = run_register(tree, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R, t, 0, rr, (char*)d_ws, ws_bytes,
                    (hipStream_t)stream, 1, d_stops, nullptr, d_bins, nullptr, loglik ? nrm : nullptr);
  if (rc) return rc;
  if (loglik) *loglik = nrm[27];
  return HGMM_OK;
}

int hgmm_normal_equations(hgmm_tree tree, const double* d_bins, int64_t n, void* d_ws, size_t ws_bytes, void* stream,
                          double H[36], double g[6]) {
  if (!tree || !d_bins || !d_ws || !H || !g) return fail(HGMM_EINVAL, "null pointer argument");
  if (tree->trees.size() != 1) return fail(HGMM_EINVAL, "single-tree handle expected");
  const int64_t nodes_total = tree->total_nodes();
  RegLayout Ly = reg_layout(n, nodes_total, 1);
  if (ws_bytes < Ly.total) return fail(HGMM_EINVAL, "workspace too small");
  char* ws = (char*)d_ws;
  hipStream_t s = (hipStream_t)stream;
  int rc = grow_stage(tree, 4096);
  if (rc) return rc;
  double* h = (double*)tree->h_stage;
  int64_t* hn = (int64_t*)(tree->h_stage + 1024);
  for (int i = 0; i < 12; ++i) h[i] = (i < 9) ? (i % 4 == 0 ? 1.0 : 0.0) : 0.0;
  *hn = n;
  double* d_out = (double*)(ws + Ly.out);
  double* d_pose0 = d_out + 28;
  int64_t* d_nmov = (int64_t*)(ws + Ly.nmov);
  HIP_TRY(hipMemcpyAsync(d_pose0, h, sizeof(double) * 12, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_nmov, hn, sizeof(int64_t), hipMemcpyHostToDevice, s));
  launch_init_pose((PoseState*)(ws + Ly.state), 1, d_pose0, d_pose0 + 9, 0, nullptr, s);
  // the kernel reads the bins without modifying them in mode 1
  launch_normal(const_cast<double*>(d_bins), nullptr, tree->d_nodes, tree->d_trees,
                (PoseState*)(ws + Ly.state), d_nmov, 1, 1, 0.0, 0.0, 1, d_out, s);
  HIP_LAUNCHED();
  double* hres = h + 16;
  HIP_TRY(hipMemcpyAsync(hres, d_out, sizeof(double) * 28, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int idx = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) { H[6 * i + j] = hres[idx]; H[6 * j + i] = hres[idx]; ++idx; }
  for (int i = 0; i < 6; ++i) g[i] = hres[21 + i];
  return HGMM_OK;
}

int hgmm_tree_info(hgmm_tree tree, int index, int* levels, int64_t* n_nodes, double origin[3], double* extent) {
  if (!tree || index < 0 || index >= (int)tree->trees.size()) return fail(HGMM_EINVAL, "bad tree index");
  TreeDev T;
  HIP_TRY(hipMemcpy(&T, tree->d_trees + index, sizeof(TreeDev), hipMemcpyDeviceToHost));
  if (levels) *levels = tree->trees[index].levels;
  if (n_nodes) *n_nodes = tree_nodes(tree->trees[index].levels);
  if (origin) for (int i = 0; i < 3; ++i) origin[i] = T.origin[i];
  if (extent) *extent = T.extent;
  return HGMM_OK;
}

int hgmm_tree_export(hgmm_tree tree, int index, hgmm_tree_host* out) {
  if (!tree || !out || index < 0 || index >= (int)tree->trees.size()) return fail(HGMM_EINVAL, "bad argument");
  const TreeHost& th = tree->trees[index];
  const int64_t nn = tree_nodes(th.levels);
  std::vector<NodeD> nd((size_t)nn);
  TreeDev T;
  HIP_TRY(hipMemcpy(nd.data(), tree->d_nodes + th.node_base, sizeof(NodeD) * nn, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(&T, tree->d_trees + index, sizeof(TreeDev), hipMemcpyDeviceToHost));
  out->levels = th.levels;
  out->n_points = th.n_points;
  for (int i = 0; i < 3; ++i) out->origin[i] = T.origin[i];
  out->extent = T.extent;
  for (int64_t g = 0; g < nn; ++g) {
    const NodeD& a = nd[g];
    if (out->live) out->live[g] = a.live;
    if (out->has_children) out->has_children[g] = a.has_children;
    if (out->count) out->count[g] = a.count;
    if (out->pi) out->pi[g] = a.pi;
    if (out->pig) out->pig[g] = a.pig;
    if (out->kappa) out->kappa[g] = a.kappa;
    for (int i = 0; i < 3; ++i) {
      if (out->mu) out->mu[3 * g + i] = a.mu[i];
      if (out->lam) out->lam[3 * g + i] = a.lam[i];
    }
    for (int i = 0; i < 6; ++i)
      if (out->cov) out->cov[6 * g + i] = a.cov[i];
    for (int i = 0; i < 9; ++i)
      if (out->evec) out->evec[9 * g + i] = a.evec[i];
  }
  return HGMM_OK;
}

int hgmm_tree_labels(hgmm_tree tree, int index, int32_t* d_labels, void* stream) {
  if (!tree || !d_labels || index < 0 || index >= (int)tree->trees.size()) return fail(HGMM_EINVAL, "bad argument");
  if (!tree->has_labels) return fail(HGMM_EINVAL, "this handle has no labels (imported tree)");
  const TreeHost& th = tree->trees[index];
  HIP_TRY(hipMemcpyAsync(d_labels, tree->d_labels + th.label_base, sizeof(int32_t) * th.levels * th.n_points,
                         hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return HGMM_OK;
}

int hgmm_tree_import(const hgmm_tree_host* in, void* stream, hgmm_tree* out) {
  if (!in || !out || !in->live || !in->has_children || !in->pi || !in->pig || !in->mu || !in->cov || !in->lam ||
      !in->evec || !in->kappa)
    return fail(HGMM_EINVAL, "null pointer argument");
  if (in->levels < 1 || in->levels > HGMM_MAX_LEVELS) return fail(HGMM_EINVAL, "levels outside [1, 6]");
  hgmm_forest_s* f = new hgmm_forest_s();
  (void)hipGetDevice(&f->device);
  f->trees.assign(1, TreeHost{in->levels, std::max<int64_t>(in->n_points, 1), 0, 0, 0});
  int rc = setup_forest(f);
  if (rc) { free_forest(f); return rc; }
  const int64_t nn = tree_nodes(in->levels);
  std::vector<NodeD> nd((size_t)nn);
  for (int64_t g = 0; g < nn; ++g) {
    NodeD& a = nd[g];
    memset(&a, 0, sizeof(a));
    a.live = in->live[g];
    a.has_children = in->has_children[g];
    a.count = in->count ? in->count[g] : 0;
    a.pi = in->pi[g];
    a.pig = in->pig[g];
    a.kappa = in->kappa[g];
    for (int i = 0; i < 3; ++i) { a.mu[i] = in->mu[3 * g + i]; a.lam[i] = in->lam[3 * g + i]; }
    for (int i = 0; i < 6; ++i) a.cov[i] = in->cov[6 * g + i];
    for (int i = 0; i < 9; ++i) a.evec[i] = in->evec[9 * g + i];
  }
  TreeDev T;
  memset(&T, 0, sizeof(T));
  for (int i = 0; i < 3; ++i) T.origin[i] = in->origin[i];
  T.extent = in->extent;
  T.levels = in->levels;
  T.n_points = (int32_t)f->trees[0].n_points;
  hipStream_t s = (hipStream_t)stream;
  auto body = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(f->d_nodes, nd.data(), sizeof(NodeD) * nn, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(f->d_trees, &T, sizeof(TreeDev), hipMemcpyHostToDevice, s));
    launch_import_nodes(f->d_nodes, f->d_tab, nn, s);
    HIP_LAUNCHED();
    HIP_TRY(hipStreamSynchronize(s));
    return HGMM_OK;
  };
  rc = body();
  if (rc) { free_forest(f); return rc; }
  f->has_labels = false;
  *out = f;
  return HGMM_OK;
}

static int check_offsets(const int64_t* offsets, int B) {
  if (!offsets || B < 1) return fail(HGMM_EINVAL, "null offsets or empty batch");
  if (offsets[0] != 0) return fail(HGMM_EINVAL, "offsets[0] must be 0");
  for (int b = 0; b < B; ++b)
    if (offsets[b + 1] < offsets[b]) return fail(HGMM_EINVAL, "offsets must be non-decreasing");
  if (offsets[B] > (int64_t)INT32_MAX / 2) return fail(HGMM_EINVAL, "too many points");
  return HGMM_OK;
}

size_t hgmm_build_batch_workspace_bytes(const int64_t* offsets, const int32_t* levels, int B) {
  if (check_offsets(offsets, B) || !levels) return 0;
  std::vector<TreeHost> t((size_t)B);
  for (int b = 0; b < B; ++b) {
    if (levels[b] < 1 || levels[b] > HGMM_MAX_LEVELS) return 0;
    t[b] = TreeHost{levels[b], offsets[b + 1] - offsets[b], 0, 0, 0};
  }
  int Lmax = 0;
  for (auto& x : t) Lmax = std::max(Lmax, x.levels);
  return build_layout(offsets[B], max_jobs_for(t), max_lvl_for(t), B, Lmax).total;
}

size_t hgmm_register_batch_workspace_bytes(hgmm_tree forest, const int64_t* offsets, int B) {
  if (!forest || check_offsets(offsets, B) || B > (int)forest->trees.size()) return 0;
  return reg_layout(offsets[B], forest->total_nodes(), B).total;
}

size_t hgmm_autotune_workspace_bytes(const int64_t* src_offsets, const int32_t* levels, const int64_t* tgt_offsets,
                                     int B) {
  const size_t b = hgmm_build_batch_workspace_bytes(src_offsets, levels, B);
  if (b == 0 || !tgt_offsets) return b;
  if (check_offsets(tgt_offsets, B)) return 0;
  int64_t nodes = 0;
  for (int i = 0; i < B; ++i) nodes += tree_nodes(levels[i]);
  return std::max(b, reg_layout(tgt_offsets[B], nodes, B).total);
}

// Forest of B trees from clouds [offsets[b], offsets[b+1]) of the SoA arrays
// in (whose stride may exceed offsets[B]).
static int build_forest(const BuildInput& in, const int64_t* offsets, const int32_t* levels, int B,
                        const hgmm_build_params* p, void* d_ws, size_t ws_bytes, void* stream, hgmm_tree* forest) {
  int rc;
  for (int b = 0; b < B; ++b) {
    if (levels[b] < 1 || levels[b] > HGMM_MAX_LEVELS) return fail(HGMM_EINVAL, "levels[%d] outside [1, 6]", b);
    if (offsets[b + 1] - offsets[b] < 8) return fail(HGMM_ETOOFEW, "cloud %d has fewer than 8 points", b);
  }
  hgmm_forest_s* f = *forest;
  const bool fresh = (f == nullptr);
  if (fresh) f = new hgmm_forest_s();
  HIP_TRY(hipGetDevice(&f->device));
  f->trees.resize((size_t)B);
  for (int b = 0; b < B; ++b) f->trees[b] = TreeHost{levels[b], offsets[b + 1] - offsets[b], 0, 0, 0};
  rc = setup_forest(f);
  if (!rc)
    rc = (g_tune.build_graph && !g_prof.on) ? run_build_graph(f, in, *p, (char*)d_ws, ws_bytes, (hipStream_t)stream)
                                            : run_build(f, in, *p, (char*)d_ws, ws_bytes, (hipStream_t)stream);
  if (rc && fresh) { free_forest(f); return rc; }
  *forest = f;
  return rc;
}

int hgmm_build_batch(const float* d_xyz, const int64_t* offsets, const int32_t* levels, int B,
                     const hgmm_build_params* p, void* d_ws, size_t ws_bytes, void* stream, hgmm_tree* forest) {
  int rc = check_build_params(p);
  if (rc) return rc;
  if ((rc = check_offsets(offsets, B))) return rc;
  if (!d_xyz || !d_ws || !forest || !levels) return fail(HGMM_EINVAL, "null pointer argument");
  const int64_t n = offsets[B];
  return build_forest(BuildInput{d_xyz, d_xyz + n, d_xyz + 2 * n}, offsets, levels, B, p, d_ws, ws_bytes, stream,
                      forest);
}

int hgmm_register_batch(hgmm_tree forest, const float* d_xyz, const int64_t* offsets, int B,
                        const hgmm_reg_params* p, const double* R0, const double* t0, const int32_t* active,
                        void* d_ws, size_t ws_bytes, void* stream, double* R, double* t, int* iters, double* loglik,
                        int* status) {
  int rc = check_offsets(offsets, B);
  if (rc) return rc;
  if (!forest || !d_xyz || !p || !d_ws || !R || !t || !iters) return fail(HGMM_EINVAL, "null pointer argument");
  if (B > (int)forest->trees.size()) return fail(HGMM_EINVAL, "batch size %d > forest size %d", B,
                                                  (int)forest->trees.size());
  if (p->max_iters < 1) return fail(HGMM_EINVAL, "max_iters must be >= 1");
  for (int b = 0; b < B; ++b)
    if (offsets[b + 1] - offsets[b] < 1) return fail(HGMM_ETOOFEW, "cloud %d to register is empty", b);
  std::vector<int64_t> offs(offsets, offsets + B + 1);
  RegRun rr{p->max_iters, p->lambda_c, p->tol_rot, p->tol_trans_rel, p->max_levels};
  std::vector<PoseState> res((size_t)B);
  const int64_t n = offsets[B];
  rc = run_register(forest, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R0, t0, 1, rr, (char*)d_ws, ws_bytes,
                    (hipStream_t)stream, 0, nullptr, nullptr, nullptr, res.data(), nullptr, active);
  if (rc) return rc;
  int worst = HGMM_OK;
  for (int b = 0; b < B; ++b) {
    for (int i = 0; i < 9; ++i) R[9 * b + i] = res[b].R[i];
    for (int i = 0; i < 3; ++i) t[3 * b + i] = res[b].t[i];
    iters[b] = res[b].iters;
    if (loglik) loglik[b] = res[b].loglik;
    if (status) status[b] = res[b].status;
    if (res[b].status != 0) worst = res[b].status;
  }
  if (worst != HGMM_OK && !status) return fail(worst, "normal equations not positive definite for some pair");
  return HGMM_OK;
}

int hgmm_register_warm_batch(hgmm_tree forest, const float* d_xyz, const int64_t* offsets, int B,
                             const hgmm_reg_params* p, int coarse_levels, int rule, const double* R0,
                             const double* t0, void* d_ws, size_t ws_bytes, void* stream, double* R, double* t,
                             int* iters, double* loglik, int* status, int32_t* fallback) {
  int rc = check_offsets(offsets, B);
  if (rc) return rc;
  if (!forest || !d_xyz || !p || !R0 || !t0 || !d_ws || !R || !t || !iters || !loglik || !status || !fallback)
    return fail(HGMM_EINVAL, "null pointer argument");
  if (B > (int)forest->trees.size()) return fail(HGMM_EINVAL, "batch size %d > forest size %d", B,
                                                  (int)forest->trees.size());
  if (p->max_iters < 1) return fail(HGMM_EINVAL, "max_iters must be >= 1");
  if (coarse_levels < 0) return fail(HGMM_EINVAL, "coarse_levels must be >= 0");
  if (rule != 0 && rule != 1) return fail(HGMM_EINVAL, "rule must be 0 (plain) or 1 (identity)");
  for (int b = 0; b < B; ++b)
    if (offsets[b + 1] - offsets[b] < 1) return fail(HGMM_ETOOFEW, "cloud %d to register is empty", b);
  std::vector<int64_t> offs(offsets, offsets + B + 1);
  const int64_t n = offsets[B];
  const float *xs = d_xyz, *ys = d_xyz + n, *zs = d_xyz + 2 * n;
  hipStream_t s = (hipStream_t)stream;
  // every run below registers the same points onto the same trees with the
  // same workspace, so the first one sorts them (reg_sort) and the others
  // reuse its order
  RegRun full{p->max_iters, p->lambda_c, p->tol_rot, p->tol_trans_rel, 0};
  std::vector<PoseState> warm((size_t)B), plain((size_t)B);
  // the start: the given transforms, refined with the capped descent
  std::vector<double> Rs(R0, R0 + 9 * (size_t)B), ts(t0, t0 + 3 * (size_t)B);
  int deepest = 0;
  for (int b = 0; b < B; ++b) deepest = std::max(deepest, forest->trees[b].levels);
  if (coarse_levels > 0 && deepest > coarse_levels) {
    const RegRun capped{p->max_iters, p->lambda_c, p->tol_rot, p->tol_trans_rel, coarse_levels};
    rc = run_register(forest, xs, ys, zs, offs, R0, t0, 1, capped, (char*)d_ws, ws_bytes, s, 0, nullptr, nullptr,
                      nullptr, warm.data(), nullptr);
    if (rc) return rc;
    full.sorted = true;
    for (int b = 0; b < B; ++b) {
      if (warm[b].status != 0) continue;
      for (int i = 0; i < 9; ++i) Rs[9 * (size_t)b + i] = warm[b].R[i];
      for (int i = 0; i < 3; ++i) ts[3 * (size_t)b + i] = warm[b].t[i];
    }
  }
  rc = run_register(forest, xs, ys, zs, offs, Rs.data(), ts.data(), 1, full, (char*)d_ws, ws_bytes, s, 0, nullptr,
                    nullptr, nullptr, warm.data(), nullptr);
  if (rc) return rc;
  full.sorted = true;
  std::vector<int32_t> fb((size_t)B, 0);
  if (rule == 0) {
    rc = run_register(forest, xs, ys, zs, offs, nullptr, nullptr, 1, full, (char*)d_ws, ws_bytes, s, 0, nullptr,
                      nullptr, nullptr, plain.data(), nullptr);
    if (rc) return rc;
    for (int b = 0; b < B; ++b)
      fb[b] = (warm[b].status != 0) || (plain[b].status == 0 && warm[b].loglik < plain[b].loglik);
  } else {
    std::vector<double> Ri(9 * (size_t)B, 0.0), ti(3 * (size_t)B, 0.0);
    for (int b = 0; b < B; ++b) Ri[9 * (size_t)b] = Ri[9 * (size_t)b + 4] = Ri[9 * (size_t)b + 8] = 1.0;
    std::vector<double> nrm(28 * (size_t)B);
    RegRun one{1, p->lambda_c, 0.0, 0.0, 0};
    one.sorted = true;
    rc = run_register(forest, xs, ys, zs, offs, Ri.data(), ti.data(), 1, one, (char*)d_ws, ws_bytes, s, 1, nullptr,
                      nullptr, nullptr, nullptr, nrm.data());
    if (rc) return rc;
    std::vector<int32_t> act((size_t)B, 0);
    bool any = false;
    for (int b = 0; b < B; ++b) {
      fb[b] = (warm[b].status != 0) || (warm[b].loglik < nrm[28 * (size_t)b + 27]);
      act[b] = fb[b];
      any = any || fb[b];
    }
    if (any) {
      rc = run_register(forest, xs, ys, zs, offs, nullptr, nullptr, 1, full, (char*)d_ws, ws_bytes, s, 0, nullptr,
                        nullptr, nullptr, plain.data(), nullptr, act.data());
      if (rc) return rc;
    }
  }
  for (int b = 0; b < B; ++b) {
    const PoseState& r = fb[b] ? plain[b] : warm[b];
    for (int i = 0; i < 9; ++i) R[9 * (size_t)b + i] = r.R[i];
    for (int i = 0; i < 3; ++i) t[3 * (size_t)b + i] = r.t[i];
    iters[b] = r.iters;
    loglik[b] = r.loglik;
    status[b] = r.status;
    fallback[b] = fb[b];
  }
  return HGMM_OK;
}

int hgmm_estep_batch(hgmm_tree forest, const float* d_xyz, const int64_t* offsets, int B, const double* R,
                     const double* t, double lambda_c, void* d_ws, size_t ws_bytes, void* stream, double* loglik,
                     int32_t* d_stop) {
  int rc = check_offsets(offsets, B);
  if (rc) return rc;
  if (!forest || !d_xyz || !d_ws || !loglik) return fail(HGMM_EINVAL, "null pointer argument");
  if (B > (int)forest->trees.size()) return fail(HGMM_EINVAL, "batch size > forest size");
  for (int b = 0; b < B; ++b)
    if (offsets[b + 1] - offsets[b] < 1) return fail(HGMM_ETOOFEW, "cloud %d is empty", b);
  std::vector<int64_t> offs(offsets, offsets + B + 1);
  RegRun rr{1, lambda_c, 0.0, 0.0, 0};
  std::vector<double> nrm(28 * (size_t)B);
  const int64_t n = offsets[B];
  rc = run_register(forest, d_xyz, d_xyz + n, d_xyz + 2 * n, offs, R, t, 1, rr, (char*)d_ws, ws_bytes,
                    (hipStream_t)stream, 1, d_stop, nullptr, nullptr, nullptr, nrm.data());
  if (rc) return rc;
  for (int b = 0; b < B; ++b) loglik[b] = nrm[28 * (size_t)b + 27];
  return HGMM_OK;
}

// ---- frame-to-frame odometry over a scan sequence -----------------------

size_t hgmm_odometry_workspace_bytes(const int64_t* offsets, int F, int levels) {
  if (F < 2 || check_offsets(offsets, F) || levels < 1 || levels > HGMM_MAX_LEVELS) return 0;
  std::vector<int32_t> lv((size_t)F - 1, levels);
  const size_t b = hgmm_build_batch_workspace_bytes(offsets, lv.data(), F - 1);
  if (b == 0) return 0;
  return std::max(b, reg_layout(offsets[F] - offsets[1], (int64_t)(F - 1) * tree_nodes(levels), F - 1).total);
}

int hgmm_odometry(const float* d_xyz, const int64_t* offsets, int F, const hgmm_build_params* bp,
                  const hgmm_reg_params* rp, const double* R0, const double* t0, int prior_restart, void* d_ws,
                  size_t ws_bytes,
                  void* stream, hgmm_tree* forest, double* R_rel, double* t_rel, double* R_abs, double* t_abs,
                  int* iters, int* status) {
  if (F < 2) return fail(HGMM_EINVAL, "a sequence needs at least 2 frames");
  int rc = check_offsets(offsets, F);
  if (rc) return rc;
  if ((rc = check_build_params(bp))) return rc;
  if (!d_xyz || !rp || !d_ws || !forest || !R_rel || !t_rel || !R_abs || !t_abs || !iters)
    return fail(HGMM_EINVAL, "null pointer argument");
  if (rp->max_iters < 1) return fail(HGMM_EINVAL, "max_iters must be >= 1");
  for (int k = 0; k < F; ++k)
    if (offsets[k + 1] - offsets[k] < 8) return fail(HGMM_ETOOFEW, "frame %d has fewer than 8 points", k);
  const size_t need = hgmm_odometry_workspace_bytes(offsets, F, bp->levels);
  if (need == 0 || ws_bytes < need) return fail(HGMM_EINVAL, "odometry workspace too small: %zu < %zu", ws_bytes, need);
  const int64_t T = offsets[F];
  // the trees of frames 0 .. F-2, every level of all of them in the same launches
  std::vector<int32_t> lv((size_t)F - 1, bp->levels);
  rc = build_forest(BuildInput{d_xyz, d_xyz + T, d_xyz + 2 * T}, offsets, lv.data(), F - 1, bp, d_ws, ws_bytes,
                    stream, forest);
  if (rc) return rc;
  // frame k+1 registered onto the tree of frame k, all pairs in one call
  const int64_t o1 = offsets[1];
  std::vector<int64_t> offs((size_t)F);
  for (int k = 0; k < F; ++k) offs[k] = offsets[k + 1] - o1;
  RegRun rr{rp->max_iters, rp->lambda_c, rp->tol_rot, rp->tol_trans_rel, rp->max_levels};
  std::vector<PoseState> res((size_t)F - 1);
  rc = run_register(*forest, d_xyz + o1, d_xyz + T + o1, d_xyz + 2 * T + o1, offs, R0, t0, 1, rr, (char*)d_ws,
                    ws_bytes, (hipStream_t)stream, 0, nullptr, nullptr, nullptr, res.data(), nullptr);
  if (rc) return rc;
  if (prior_restart && F > 2) {
    // second start of every pair from the neighbouring pair's motion (the
    // frame before; pair 0 from pair 1), all pairs in one call; each pair
    // keeps the run that ends with the higher log-likelihood
    std::vector<double> Rp(9 * (size_t)(F - 1)), tp(3 * (size_t)(F - 1));
    for (int k = 0; k < F - 1; ++k) {
      const PoseState& S = res[(size_t)(k == 0 ? 1 : k - 1)];
      for (int i = 0; i < 9; ++i) Rp[9 * (size_t)k + i] = S.R[i];
      for (int i = 0; i < 3; ++i) tp[3 * (size_t)k + i] = S.t[i];
    }
    std::vector<PoseState> res2((size_t)F - 1);
    rc = run_register(*forest, d_xyz + o1, d_xyz + T + o1, d_xyz + 2 * T + o1, offs, Rp.data(), tp.data(), 1, rr,
                      (char*)d_ws, ws_bytes, (hipStream_t)stream, 0, nullptr, nullptr, nullptr, res2.data(), nullptr);
    if (rc) return rc;
    for (int k = 0; k < F - 1; ++k) {
      const PoseState& a = res[(size_t)k];
      const PoseState& b = res2[(size_t)k];
      if (b.status == 0 && (a.status != 0 || b.loglik > a.loglik)) res[(size_t)k] = b;
    }
  }
  // chain: frame-0 coordinates = R_abs[k] (frame-k coordinates) + t_abs[k]
  for (int i = 0; i < 9; ++i) R_abs[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int i = 0; i < 3; ++i) t_abs[i] = 0.0;
  int worst = HGMM_OK;
  for (int k = 1; k < F; ++k) {
    const PoseState& S = res[(size_t)k - 1];
    double* Rr = R_rel + 9 * (size_t)(k - 1);
    double* tr = t_rel + 3 * (size_t)(k - 1);
    for (int i = 0; i < 9; ++i) Rr[i] = S.R[i];
    for (int i = 0; i < 3; ++i) tr[i] = S.t[i];
    iters[k - 1] = S.iters;
    if (status) status[k - 1] = S.status;
    if (S.status != 0) worst = S.status;
    const double* Rp = R_abs + 9 * (size_t)(k - 1);
    const double* tp = t_abs + 3 * (size_t)(k - 1);
    double* Ra = R_abs + 9 * (size_t)k;
    double* ta = t_abs + 3 * (size_t)k;
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) Ra[3 * i + j] = Rp[3 * i] * Rr[j] + Rp[3 * i + 1] * Rr[3 + j] + Rp[3 * i + 2] * Rr[6 + j];
      ta[i] = Rp[3 * i] * tr[0] + Rp[3 * i + 1] * tr[1] + Rp[3 * i + 2] * tr[2] + tp[i];
    }
  }
  if (worst != HGMM_OK && !status) return fail(worst, "normal equations not positive definite for some frame pair");
  return HGMM_OK;
}

void hgmm_tree_destroy(hgmm_tree tree) { free_forest(tree); }

}  // extern "C"
