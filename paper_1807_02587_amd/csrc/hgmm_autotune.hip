// Autotuner of the launch shapes (hgmm_tuning) for one workload.
//
// The construction of a level can run a parent in one block for all EM
// iterations (three block sizes) or cut it into tiles with one launch per
// iteration; which is faster depends on how many parents a level has and how
// their sizes are spread, i.e. on the workload.  The tuner times the caller's
// own batch (construction, and registration when target clouds are given)
// under candidate settings with HIP events on the caller's stream, by
// coordinate descent over the knobs, and leaves the fastest setting in effect.
// A build_graph = 1 or 2 candidate is timed after two untimed runs (the first
// construction of a shape is host-planned and records the work counts, the
// second captures the graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/hgmm.h"
#include "hgmm_internal.h"

namespace {

struct Knob {
  int32_t hgmm_tuning::*field;
  std::vector<int32_t> cand;
};

const std::vector<Knob>& knobs() {
  static const std::vector<Knob> k = {
      {&hgmm_tuning::block64_max, {0, 128, 256, 512}},
      {&hgmm_tuning::block256_max, {256, 512, 1024, 2048}},
      {&hgmm_tuning::block512_max, {1024, 2048, 4096, 8192}},
      {&hgmm_tuning::tile_threads, {256, 512, 1024}},
      {&hgmm_tuning::min_tile, {256, 512, 1024, 2048, 4096}},
      {&hgmm_tuning::target_tiles, {256, 512, 1024, 2048, 4096}},
      {&hgmm_tuning::max_tile, {1024, 2048, 4096, 8192, 16384}},
      {&hgmm_tuning::reg_tile, {256, 512, 1024, 2048}},
      {&hgmm_tuning::reg_chunk, {2, 4, 8, 16}},
      {&hgmm_tuning::reg_graph, {0, 1}},
      {&hgmm_tuning::reg_sort, {0, 1}},
      {&hgmm_tuning::reg_lds_levels, {2, 3}},
      {&hgmm_tuning::build_graph, {0, 1, 2}},
      {&hgmm_tuning::fold_tiles, {0, 256, 1024, 4096, 1 << 30}},
  };
  return k;
}

struct Workload {
  const float* d_src;
  const int64_t* src_off;
  const int32_t* levels;
  int B;
  const float* d_tgt;
  const int64_t* tgt_off;
  const hgmm_build_params* bp;
  const hgmm_reg_params* rp;
  void* ws;
  size_t ws_bytes;
  hipStream_t s;
};

// One timed run (construction, then registration from the identity); ms < 0
// when the setting fails.
int run_once(const Workload& w, hgmm_tree* forest, hipEvent_t e0, hipEvent_t e1, double* ms) {
  std::vector<double> R(9 * (size_t)w.B), t(3 * (size_t)w.B), ll((size_t)w.B);
  std::vector<int> iters((size_t)w.B), st((size_t)w.B);
  if (hipEventRecord(e0, w.s) != hipSuccess) return hgmm_fail(HGMM_EHIP, "event record failed");
  int rc = hgmm_build_batch(w.d_src, w.src_off, w.levels, w.B, w.bp, w.ws, w.ws_bytes, w.s, forest);
  if (rc) return rc;
  if (w.d_tgt) {
    rc = hgmm_register_batch(*forest, w.d_tgt, w.tgt_off, w.B, w.rp, nullptr, nullptr, nullptr, w.ws, w.ws_bytes, w.s,
                             R.data(), t.data(), iters.data(), ll.data(), st.data());
    if (rc) return rc;
  }
  if (hipEventRecord(e1, w.s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return hgmm_fail(HGMM_EHIP, "event synchronisation failed");
  float f = 0.f;
  if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return hgmm_fail(HGMM_EHIP, "event timing failed");
  *ms = f;
  return HGMM_OK;
}

int measure(const Workload& w_, const hgmm_tuning& tu, int reps, hgmm_tree* forest, hipEvent_t e0, hipEvent_t e1,
            double* best) {
  const Workload& w = w_;
  int rc = hgmm_set_tuning(&tu);
  if (rc) return rc;
  if (tu.build_graph) {
    // a graph construction of a new shape first runs host-planned (recording
    // the work counts), then captures: time only the replays
    for (int w = 0; w < 2; ++w) {
      double ms = 0.0;
      if ((rc = run_once(w_, forest, e0, e1, &ms))) return rc;
    }
  }
  double m = 1e300;
  for (int r = 0; r < reps; ++r) {
    double ms = 0.0;
    if ((rc = run_once(w, forest, e0, e1, &ms))) return rc;
    m = std::min(m, ms);
  }
  *best = m;
  return HGMM_OK;
}

}  // namespace

extern "C" int hgmm_autotune(const float* d_src, const int64_t* src_offsets, const int32_t* levels, int B,
                             const float* d_tgt, const int64_t* tgt_offsets, const hgmm_build_params* bp,
                             const hgmm_reg_params* rp, void* d_ws, size_t ws_bytes, void* stream, int reps,
                             int passes, hgmm_tuning* best, double* best_ms, double* start_ms) {
  if (!d_src || !src_offsets || !levels || B < 1 || !bp || !d_ws || !best)
    return hgmm_fail(HGMM_EINVAL, "null pointer argument or empty batch");
  if (d_tgt && (!tgt_offsets || !rp)) return hgmm_fail(HGMM_EINVAL, "target clouds need offsets and parameters");
  if (reps < 1 || reps > 16 || passes < 1 || passes > 4) return hgmm_fail(HGMM_EINVAL, "reps in [1,16], passes in [1,4]");
  const size_t need_b = hgmm_build_batch_workspace_bytes(src_offsets, levels, B);
  if (need_b == 0) return hgmm_fail(HGMM_EINVAL, "invalid offsets or levels");
  if (ws_bytes < need_b) return hgmm_fail(HGMM_EINVAL, "workspace too small for the construction");
  Workload w{d_src, src_offsets, levels, B, d_tgt, tgt_offsets, bp, rp, d_ws, ws_bytes, (hipStream_t)stream};
  hgmm_tuning start;
  hgmm_get_tuning(&start);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hgmm_fail(HGMM_EHIP, "event creation failed");
  }
  hgmm_tree forest = nullptr;
  int rc = HGMM_OK;
  hgmm_tuning cur = start;
  double cur_ms = 0.0;
  // the registration workspace needs the forest: build once with the start setting
  rc = measure(w, cur, 1, &forest, e0, e1, &cur_ms);
  if (!rc && d_tgt) {
    const size_t need_r = hgmm_register_batch_workspace_bytes(forest, tgt_offsets, B);
    if (need_r == 0 || ws_bytes < need_r) rc = hgmm_fail(HGMM_EINVAL, "workspace too small for the registration");
  }
  if (!rc) rc = measure(w, cur, reps, &forest, e0, e1, &cur_ms);
  if (start_ms) *start_ms = cur_ms;
  for (int pass = 0; pass < passes && !rc; ++pass) {
    bool moved = false;
    for (const Knob& k : knobs()) {
      for (int32_t v : k.cand) {
        if (cur.*k.field == v) continue;
        hgmm_tuning t = cur;
        t.*k.field = v;
        if (hgmm_set_tuning(&t) != HGMM_OK) continue;  // inconsistent combination: skip it
        double ms = 0.0;
        if ((rc = measure(w, t, reps, &forest, e0, e1, &ms))) break;
        if (ms < cur_ms * 0.99) { cur = t; cur_ms = ms; moved = true; }
      }
      if (rc) break;
    }
    if (!moved) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (forest) hgmm_tree_destroy(forest);
  if (rc) {
    hgmm_set_tuning(&start);
    return rc;
  }
  hgmm_set_tuning(&cur);
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return HGMM_OK;
}
