// Host-side declarations of the kernel launchers (one translation unit per
// kernel family; the C ABI in hgmm_api.hip drives them).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hgmm_dev.h"

namespace hgmm {

void launch_fill_u32(void* p, uint32_t v, int64_t n_words, hipStream_t s);

// build.  With a device count (dn, dntiles, dnjobs: a level planned on the
// device) the kernels read their number of work items from it and the count
// given as an int is the fixed grid; with nullptr it is the number of items.
// em_block / em_mstep take their jobs from job_ids + *doff when doff is given.
void launch_root(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles, const Job* jobs,
                 int njobs, TreeDev* trees, double* partials, size_t pstride, double eps, hipStream_t s,
                 const int* dntiles = nullptr, const int* dnjobs = nullptr);
void launch_init_children(const Job* jobs, int njobs, const TreeDev* trees, NodeD* nodes, NodeF* tab, double eps,
                          hipStream_t s, const int* dn = nullptr);
// one EM iteration of the tiled jobs (iteration 0: first = 1).  inline_fold:
// every tile block folds the previous iteration's partials (part_prev) and
// runs the M-step from ch_prev, the job's first tile publishing the children
// in ch_next (ping-pong between iterations); otherwise the blocks read the
// frames written by launch_em_fold (kFrameBytes per tiled job), which between
// two iterations folds the partials and runs the M-step once per tiled job
// (children ch updated in place, next frames written).  After the last
// iteration, the final M-step from that iteration's children (chsrc, one set
// of 8 per tiled job) writes the node records.
constexpr size_t kFrameBytes = 512;
void launch_em_tile(int nt, const float* xs, const float* ys, const float* zs, const Tile* tiles, const int* tile_ids,
                    int n, const Job* jobs, const NodeF* tab, const NodeF* ch_prev, NodeF* ch_next, const void* frames,
                    const double* part_prev, double* part_next, size_t pstride, double eps, double min_mass,
                    int first, bool inline_fold, hipStream_t s, const int* dn = nullptr);
void launch_em_fold(const int* job_ids, int n, const Job* jobs, const double* partials, size_t pstride, double eps,
                    double min_mass, NodeF* ch, void* frames, hipStream_t s, const int* dn = nullptr,
                    const int* doff = nullptr);
void launch_em_mstep(const int* job_ids, int n, const Job* jobs, NodeF* tab, NodeD* nodes, const double* partials,
                     size_t pstride, double eps, double min_mass, const NodeF* chsrc, hipStream_t s,
                     const int* dn = nullptr, const int* doff = nullptr);
// all EM iterations of n jobs, one block of nt (64, 256 or 512) threads per job
void launch_em_block(int nt, const float* xs, const float* ys, const float* zs, const int* job_ids, int n,
                     const Job* jobs, NodeF* tab, NodeD* nodes, int iters, double eps, double min_mass,
                     hipStream_t s, const int* dn = nullptr, const int* doff = nullptr);
void launch_partition(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                      const Job* jobs, const NodeF* tab, const NodeD* nodes, uint8_t* child, int* tile_counts,
                      hipStream_t s, const int* dn = nullptr);
void launch_prefix(const Job* jobs, int njobs, const int* tile_counts, int* tile_base, NodeD* nodes, int2* lvl_info,
                   hipStream_t s, const int* dn = nullptr);
void launch_scatter(const float* xs, const float* ys, const float* zs, const int* perm, const Tile* tiles, int ntiles,
                    const Job* jobs, const TreeDev* trees, const uint8_t* child, const int* tile_base, float* xo,
                    float* yo, float* zo, int* perm_out, int32_t* labels, int level, int64_t level_off,
                    hipStream_t s, const int* dn = nullptr);
void launch_finalize_level(const Job* jobs, int njobs, NodeD* nodes, NodeF* tab, hipStream_t s,
                           const int* dn = nullptr);

// the plan of one level on the device (jobs, class-ordered job ids, tiles,
// tile ids of the tiled jobs, and the PlanField counts in plan)
void launch_plan_level(const LevelTree* lt, int nlt, int per, int level, int64_t loff_prev, int64_t loff_cur,
                       const int2* lvl_prev, const TreeDev* trees, int b64, int b256, int b512, int target_tiles,
                       int min_tile, int max_tile, int max_jobs, int max_tiles, Job* jobs, int* job_ids, Tile* tiles,
                       int* tile_ids, int* plan, hipStream_t s);

// registration
void launch_set_stop_flags(NodeF* tab, const NodeD* nodes, int64_t n, double lambda_c, hipStream_t s);
void launch_init_pose(PoseState* st, int npairs, const double* R0, const double* t0, int stride, const int* active,
                      hipStream_t s);
// perm (nullable): original index of each point when the cloud was reordered,
// for the per-point outputs stop_out / gamma_out
// grid: 8 * ceil(ntiles / 8) blocks in XCD-aware tile order; fbins receives
// the fixed-point moments, or, when atomic_bins is given, the moments are
// added to those FP64 bins with FP64 atomics instead; work (nullable): points
// processed and levels scored
// the descent's copy of the scoring records (dead nodes score -inf) with
// this call's stop flags
void launch_reg_table(const NodeF* tab, const NodeD* nodes, NodeR* rt, int64_t n, double lambda_c, hipStream_t s);
void launch_descend(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                    const TreeDev* trees, const NodeR* rtab, const PoseState* st, FixBin* fbins,
                    double* atomic_bins, int32_t* stop_out, float* gamma_out, const int* perm, int lds_levels, int max_levels,
                    unsigned long long* work, hipStream_t s);
void launch_flat_table(const NodeF* tab, const NodeD* nodes, NodeR* fr, int64_t n, hipStream_t s);
void launch_flat_estep(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                       int tile_points, const TreeDev* trees, const NodeR* ftab, const PoseState* st, double* bins,
                       int32_t* stop_out, float* gamma_out, const int* perm, int level, hipStream_t s);
void launch_soft_estep(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                       int tile_points, int max_levels, const TreeDev* trees, const NodeF* tab, const NodeD* nodes,
                       const PoseState* st, double* bins, float tau, int32_t* stops_out, const int* perm,
                       hipStream_t s);
void launch_point_loglik(const float* xs, const float* ys, const float* zs, int64_t n, const int32_t* stop,
                         const TreeDev* trees, const NodeD* nodes, const PoseState* st, float* out, hipStream_t s);
void launch_fold_bins(const TreeDev* trees, const FixBin* fbins, double* bins, int npairs, hipStream_t s);
void launch_normal(double* bins, FixBin* fbins, const NodeD* nodes, const TreeDev* trees, PoseState* st,
                   const int64_t* n_moving, int npairs, int mode, double tol_rot, double tol_trans_rel, int max_iters,
                   double* out, hipStream_t s);
int normal_values();

// spatial ordering of the moving clouds (Morton order inside each pair)
size_t sort_temp_bytes(int64_t n, int npairs);
hipError_t launch_sort_points(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                              const TreeDev* trees, int npairs, int64_t n, uint64_t* keys, uint64_t* keys_out,
                              int* vals, int* perm, void* temp, size_t temp_bytes, float* xo, float* yo, float* zo,
                              hipStream_t s);

// import / export
void launch_import_nodes(NodeD* nodes, NodeF* tab, int64_t n, hipStream_t s);

}  // namespace hgmm
