/*
 * hgmm -- GMM-Tree point cloud registration on AMD Instinct MI355X (gfx950).
 *
 * The method is Eckart, Kim, Kautz, "Fast and Accurate Point Cloud Registration
 * using Trees of Gaussian Mixtures" (2018).  Given a model cloud Z1 and a cloud
 * Z2, find the rigid T = (R, t) that maximises the likelihood of T(Z2) under a
 * mixture model of Z1 (Sec. 3, Eq. 1-2).  Two entry points carry the method:
 *
 *   hgmm_build     builds the tree of 8-component Gaussian mixtures of Z1
 *                  (Sec. 3 end, Sec. 4.1: every component owns an 8-component
 *                  child mixture; construction = per-parent EM, Eq. 2-3, run for
 *                  all parents of a level at once);
 *   hgmm_register  runs the registration EM on that tree: the adaptive
 *                  max-likelihood descent with the complexity stop
 *                  (Sec. 4.1, Algorithm 1), moment accumulation (Eq. 9) and the
 *                  PCA-form Mahalanobis least squares (Sec. 4.2, Eq. 10-16).
 *
 * Every computation runs in HIP kernels on the device.  The library never
 * falls back to the host.
 *
 * Conventions shared by every entry point
 *   - Points are FP32 SoA in device memory: x[n], y[n], z[n] back to back
 *     (one allocation of 3n floats).  The caller owns them; the library never
 *     keeps a pointer past the call.
 *   - A rigid transform maps a point p of Z2 to R p + t; R is row-major 3x3
 *     (9 doubles), t is 3 doubles, both in host memory.
 *   - Tree levels are numbered from 0; level l holds 8^(l+1) nodes and node k
 *     of level l has children 8k..8k+7 at level l+1.  (The paper numbers
 *     recursion levels from 1: its "level 2" with J = 64 is level index 1.)
 *     Nodes are stored level-major; level l of a tree starts at
 *     hgmm_level_offset(l).
 *   - A covariance is packed as [xx, xy, xz, yy, yz, zz] and includes the
 *     regularisation reg_eps * I.
 *   - "stream" is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it.  hgmm_build synchronises it once per tree level (to plan
 *     the next level's tiles); hgmm_register synchronises it once at the end
 *     to return the pose.
 *   - Workspaces are caller-owned device memory of at least the size the
 *     matching *_workspace_bytes() call returns; their contents need not be
 *     initialised.  One workspace must not be used by two calls at once.
 *   - Every int-returning function returns HGMM_OK (0) or a negative
 *     hgmm_status; hgmm_last_error() then describes the failure (thread-local).
 *     No C++ exception crosses the boundary.
 */
#ifndef HGMM_H
#define HGMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HGMM_MAX_LEVELS 6

typedef enum {
  HGMM_OK = 0,
  HGMM_EINVAL = -1,     /* bad argument: null pointer, levels outside [1, 6], workspace too small */
  HGMM_ETOOFEW = -2,    /* fewer than 8 model points, or an empty cloud to register */
  HGMM_ENONFINITE = -3, /* a non-finite coordinate in the model cloud */
  HGMM_ENOMEM = -4,     /* device or pinned-host allocation failed */
  HGMM_EHIP = -5,       /* a HIP runtime call failed */
  HGMM_ESINGULAR = -6   /* the 6x6 normal equations were not positive definite, even damped */
} hgmm_status;

/* Opaque handle to one or more device-resident trees (a forest; a single
 * build makes a forest of one tree).  It owns its node arrays, per-point
 * labels and a small pinned staging area; free it with hgmm_tree_destroy. */
typedef struct hgmm_forest_s *hgmm_tree;

/* Tree construction parameters.  The paper delegates construction to its
 * reference [33]; these are the knobs of this library's reading of it:
 * PCA-octant initialisation of each parent's 8 children, build_iters EM
 * iterations per parent, hard partition of the points by their most likely
 * child, covariance regularisation reg_eps * I, and children whose soft mass
 * falls below min_mass dropped for the rest of the build. */
typedef struct {
  int32_t levels;      /* 1..6 */
  int32_t build_iters; /* EM iterations per level, default 30 */
  double reg_eps;      /* default 1e-6 (squared length units) */
  double min_mass;     /* default 1.0 */
} hgmm_build_params;

/* Registration parameters (Sec. 4.1-4.2).  lambda_c is the complexity
 * threshold of Algorithm 1 (the paper uses 0.01; 0 gives the "GMM-Tree Ln"
 * variant of Sec. 5).  The loop stops after max_iters E/M iterations or once
 * the angle of the rotation increment is below tol_rot (radians) and the norm
 * of the translation increment is below tol_trans_rel times the model's
 * bounding-box diagonal.  max_levels > 0 caps the descent at that many levels
 * (level max_levels-1 acts as the last level, as in a tree built with
 * max_levels levels); 0 uses every level of the tree. */
typedef struct {
  int32_t max_iters;   /* default 30 */
  int32_t max_levels;  /* default 0 (all levels) */
  double lambda_c;     /* default 0.01 */
  double tol_rot;      /* default 1e-6 */
  double tol_trans_rel;/* default 1e-6 */
} hgmm_reg_params;

/* Host copy of one tree in FP64.  The caller allocates every array with
 * hgmm_tree_nodes(levels) entries (times the per-node width) before calling
 * hgmm_tree_export, or fills them before calling hgmm_tree_import. */
typedef struct {
  int32_t levels;
  int32_t pad_;
  int64_t n_points;     /* model cloud size */
  double origin[3];     /* model mean: centre of the rotation increments */
  double extent;        /* model bounding-box diagonal */
  int32_t *live;        /* 1 if the node exists */
  int32_t *has_children;/* 1 if at least one child is live */
  int64_t *count;       /* size of the node's hard partition of Z1 */
  double *pi;           /* weight inside its sibling group */
  double *pig;          /* product of weights from the root */
  double *mu;           /* 3 per node */
  double *cov;          /* 6 per node */
  double *lam;          /* 3 per node, lam1 >= lam2 >= lam3 */
  double *evec;         /* 9 per node, row a is the eigenvector of lam_a (largest-|.| entry positive) */
  double *kappa;        /* lam3 / (lam1 + lam2 + lam3), the complexity of Sec. 4.1 */
} hgmm_tree_host;

/* Defaults: levels 2, build_iters 30, reg_eps 1e-6, min_mass 1; max_iters 30,
 * lambda_c 0.01, tol_rot 1e-6, tol_trans_rel 1e-6.  Either pointer may be NULL. */
int hgmm_params_default(hgmm_build_params *bp, hgmm_reg_params *rp);

/* Nodes of a tree with `levels` levels: (8^(levels+1) - 8) / 7.  Returns -1 for
 * levels outside [1, 6]. */
int64_t hgmm_tree_nodes(int levels);
/* First node of level `level` inside a tree: (8^(level+1) - 8) / 7. */
int64_t hgmm_level_offset(int level);

/* Workspace sizes in bytes for a cloud of n points and a tree of `levels`. */
size_t hgmm_build_workspace_bytes(int64_t n, int levels);
size_t hgmm_register_workspace_bytes(int64_t n, int levels);

/* Builds the tree of d_xyz (n points, SoA FP32, device).  If *tree is NULL a
 * new handle is allocated; otherwise the handle is reused (and grown if it is
 * too small) so that repeated builds do not allocate.  Errors: HGMM_EINVAL,
 * HGMM_ETOOFEW (n < 8), HGMM_ENONFINITE, HGMM_ENOMEM, HGMM_EHIP. */
int hgmm_build(const float *d_xyz, int64_t n, const hgmm_build_params *p, void *d_ws, size_t ws_bytes,
               void *stream, hgmm_tree *tree);

/* Registers d_xyz (n points, SoA FP32, device) onto tree (tree index 0).
 * R0/t0 (host, nullable = identity / zero) is the initial transform.  On
 * return R, t hold the estimate, *iters the number of E/M iterations run
 * (== max_iters when the tolerance was not reached, which is not an error),
 * *loglik (nullable) the mean log-likelihood of the points under the nodes
 * they stopped at, from the last E-step.  HGMM_ESINGULAR leaves R, t at the
 * last good value.  Synchronises `stream` once. */
int hgmm_register(hgmm_tree tree, const float *d_xyz, int64_t n, const hgmm_reg_params *p, const double *R0,
                  const double *t0, void *d_ws, size_t ws_bytes, void *stream, double R[9], double t[3],
                  int *iters, double *loglik);

/* ---- allocation-free registration ---------------------------------------
 * For callers that cannot allocate device or pinned host memory (code under
 * stream capture, tight serving loops, harnesses that forbid it): the same
 * registration as hgmm_register (same kernels, arguments and outputs) with
 * its workspace in a static device array of HGMM_NOALLOC_SCRATCH_BYTES that
 * the library holds on every device it runs on until the process ends, and
 * its host staging in a static host buffer.  The call allocates nothing: no
 * hipMalloc, no pinned allocation, no graph (it never takes the registration
 * graph path of hgmm_tuning.reg_graph) and no profiling events.  The caller
 * still owns d_xyz and the tree; the tree itself comes from hgmm_build.
 * The scratch is looked up once per device on the first call made with that
 * device current.  Every call on one device shares that device's scratch and
 * the process-wide host staging: calls that overlap in time (two host
 * threads, or two streams) race and must be serialised by the caller.  The
 * scratch keeps the last call's contents; each call clears what it
 * accumulates into.  Errors: those of hgmm_register, plus HGMM_EINVAL when the
 * cloud and tree need more than HGMM_NOALLOC_SCRATCH_BYTES of workspace
 * (hgmm_register_workspace_bytes(n, levels) tells; about 2^19 points on a
 * 5-level tree fit).  Synchronises `stream` once per chunk of iterations. */
#define HGMM_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
#define HGMM_NOALLOC_MAX_DEVICES 64
size_t hgmm_noalloc_scratch_bytes(void);
int hgmm_register_noalloc(hgmm_tree tree, const float *d_xyz, int64_t n, const hgmm_reg_params *p,
                          const double *R0, const double *t0, void *stream, double R[9], double t[3], int *iters,
                          double *loglik);

/* One registration E-step at a fixed transform (Algorithm 1): for each point
 * the stop node (global node id inside the tree, device int32, nullable) and
 * its weight gamma (device float, nullable); per node the moments
 * d_bins[node * 6 + {0..5}] = {M0 = sum gamma, D = sum gamma (T(p) - mu_node)
 * (3 values), number of points, sum of squared Mahalanobis distances}
 * (device double, nullable), and the mean log-likelihood (host, nullable).
 * Synchronises `stream` when loglik is requested. */
int hgmm_estep(hgmm_tree tree, const float *d_xyz, int64_t n, const double R[9], const double t[3],
               double lambda_c, void *d_ws, size_t ws_bytes, void *stream, int32_t *d_stop_node,
               float *d_gamma, double *d_bins, double *loglik);

/* ---- single-level variant ("GMM J=n", Sec. 5 list of variants) ---------
 * The live nodes of tree level `level` (0 <= level < the tree's levels;
 * J = 8^(level+1) components) form one fixed-complexity mixture with their
 * global weights; every point is scored against all J components (no tree,
 * no complexity threshold), assigned to the most likely one (the lowest node
 * index on an exact tie) with its posterior among all of them as the weight,
 * and the moments drive the same PCA-form M-step (Eq. 11-16).  Outputs,
 * workspace (hgmm_register_workspace_bytes), ownership and synchronisation
 * are those of hgmm_register / hgmm_estep; the stop node is -1 for a point
 * when the level has no live node; p->lambda_c and p->max_levels are
 * ignored.  Errors: HGMM_EINVAL (null pointer, level out of range, more than
 * one tree in the handle, workspace too small), HGMM_ETOOFEW (n < 1),
 * HGMM_ESINGULAR, HGMM_EHIP. */
int hgmm_register_flat(hgmm_tree tree, const float *d_xyz, int64_t n, int level, const hgmm_reg_params *p,
                       const double *R0, const double *t0, void *d_ws, size_t ws_bytes, void *stream, double R[9],
                       double t[3], int *iters, double *loglik);
int hgmm_estep_flat(hgmm_tree tree, const float *d_xyz, int64_t n, int level, const double R[9], const double t[3],
                    void *d_ws, size_t ws_bytes, void *stream, int32_t *d_stop_node, float *d_gamma,
                    double *d_bins, double *loglik);

/* ---- queries for other consumers of the tree (Sec. 6) -------------------
 * The log density of every point of d_xyz (n points, SoA FP32, device) under
 * the tree at the node the adaptive descent of Algorithm 1 stops at (lambda_c
 * as in hgmm_reg_params), after the transform T(p) = R p + t (host R, t):
 * d_loglik[i] = log pi^g - log|cov| / 2 - d_M^2 / 2 - 3/2 log 2 pi (device
 * float, -inf for a point with no live node), and the stop node in d_node
 * (device int32, nullable; node index inside the tree).  The mean of d_loglik
 * is hgmm_estep's log-likelihood.  For scoring a scan against a map tree
 * (loop closure) or per-point occupancy.  Workspace:
 * hgmm_register_workspace_bytes.  Asynchronous on `stream`.  Errors:
 * HGMM_EINVAL (null pointer, more than one tree, workspace too small),
 * HGMM_ETOOFEW (n < 1), HGMM_EHIP. */
int hgmm_point_loglik(hgmm_tree tree, const float *d_xyz, int64_t n, const double R[9], const double t[3],
                      double lambda_c, void *d_ws, size_t ws_bytes, void *stream, int32_t *d_node, float *d_loglik);

/* ---- soft multi-path E-step (Sec. 4.1, logarithmic search) --------------
 * A point's expectation of a node is the product of its posteriors among the
 * siblings along the path from the root (a parent's expectation is the sum
 * of its children's).  Every branch whose expectation is at least tau
 * (0 < tau < 1) is followed and a branch below tau is pruned with its
 * subtree; a followed node that stops by Algorithm 1's rule (complexity <=
 * lambda_c, no live children, or the last level) receives the point with its
 * expectation E as the weight.  Per-node moments in the hgmm_estep layout
 * with the expectation-weighted count and distance sum: {sum E, sum E (T(p) -
 * mu_node) (3), sum E, sum E d_M^2}; the log-likelihood is the E-weighted mean
 * log density.  d_stops (device int32, nullable) receives the number of nodes
 * each point reached.  Registration runs the same M-step (Eq. 11-16).
 * Outputs, workspace (hgmm_register_workspace_bytes), ownership and
 * synchronisation as hgmm_register / hgmm_estep.  Errors: HGMM_EINVAL (null
 * pointer, tau outside (0, 1), more than one tree in the handle, workspace too
 * small), HGMM_ETOOFEW (n < 1), HGMM_ESINGULAR, HGMM_EHIP. */
int hgmm_register_soft(hgmm_tree tree, const float *d_xyz, int64_t n, double tau, const hgmm_reg_params *p,
                       const double *R0, const double *t0, void *d_ws, size_t ws_bytes, void *stream, double R[9],
                       double t[3], int *iters, double *loglik);
int hgmm_estep_soft(hgmm_tree tree, const float *d_xyz, int64_t n, double tau, const double R[9], const double t[3],
                    double lambda_c, void *d_ws, size_t ws_bytes, void *stream, int32_t *d_stops, double *d_bins,
                    double *loglik);

/* The PCA-form normal equations (Eq. 11-16) of one M-step from per-node
 * moments in the hgmm_estep layout (device): H (6x6 row-major, host) and g
 * (6, host) with H x = g for the increment x = (omega, tau) of
 * T(p) -> p + omega x (p - origin) + tau.  Synchronises `stream`. */
int hgmm_normal_equations(hgmm_tree tree, const double *d_bins, int64_t n, void *d_ws, size_t ws_bytes,
                          void *stream, double H[36], double g[6]);

/* ---- batched form: many uneven clouds in one call ----------------------
 * Clouds are concatenated CSR-style into one SoA buffer of offsets[B] points
 * (x[total], y[total], z[total]); cloud b occupies [offsets[b], offsets[b+1])
 * (offsets and levels are host arrays, offsets[0] = 0).  Every level of every
 * tree is fitted by the same kernel launches; the forest handle holds B trees
 * (tree b built from cloud b with levels[b] levels; p->levels is ignored).
 * hgmm_register_batch registers target cloud b onto tree b of the forest
 * for b < B (same CSR layout, its own offsets; the forest may hold more than
 * B trees, and the others are not used), starting from R0[9 b..], t0[3 b..]
 * (host, nullable = identity); active (host, nullable) skips pairs whose
 * flag is 0 (their outputs are R0, t0 and 0 iterations).  Returns per pair R (B x 9), t (B x 3),
 * iters, loglik (nullable) and status (nullable; with status NULL a singular
 * pair makes the call return HGMM_ESINGULAR).  Both synchronise `stream`. */
size_t hgmm_build_batch_workspace_bytes(const int64_t *offsets, const int32_t *levels, int B);
int hgmm_build_batch(const float *d_xyz, const int64_t *offsets, const int32_t *levels, int B,
                     const hgmm_build_params *p, void *d_ws, size_t ws_bytes, void *stream, hgmm_tree *forest);
size_t hgmm_register_batch_workspace_bytes(hgmm_tree forest, const int64_t *offsets, int B);
int hgmm_register_batch(hgmm_tree forest, const float *d_xyz, const int64_t *offsets, int B,
                        const hgmm_reg_params *p, const double *R0, const double *t0, const int32_t *active,
                        void *d_ws, size_t ws_bytes, void *stream, double *R, double *t, int *iters, double *loglik,
                        int *status);
/* Mean log-likelihood of every target cloud at a fixed transform (R: B x 9,
 * t: B x 3, host): one E-step (Algorithm 1) per pair.  d_stop (nullable,
 * device, offsets[B] int32) receives each point's stop node (index inside its
 * pair's tree, -1 if unassigned).  As for hgmm_register_batch, cloud b goes
 * with tree b and B may be below the forest size. */
int hgmm_estep_batch(hgmm_tree forest, const float *d_xyz, const int64_t *offsets, int B, const double *R,
                     const double *t, double lambda_c, void *d_ws, size_t ws_bytes, void *stream, double *loglik,
                     int32_t *d_stop);

/* ---- frame-to-frame odometry over a scan sequence ----------------------
 * The paper's LiDAR experiment (Sec. 6): successive sweeps are registered
 * frame to frame and the transforms are concatenated into a trajectory (no
 * loop closure, so errors accumulate as drift).  Frames are concatenated
 * CSR-style into one SoA buffer of offsets[F] points (x[total], y[total],
 * z[total]; host offsets, offsets[0] = 0, every frame >= 8 points).  One call
 * builds the trees of frames 0 .. F-2 as one forest (bp->levels each; the
 * handle in *forest is created or reused, tree k is frame k's model) and
 * registers frame k+1 onto tree k for every k in one batched call, starting
 * from R0[9 k..], t0[3 k..] (host, nullable = identity).  With
 * prior_restart = 1 (and F > 2) every pair is registered a second time in one
 * more batched call, started from the neighbouring pair's result (pair k from
 * pair k-1's transform, the motion of the frame before; pair 0 from pair
 * 1's), and keeps whichever run ends with the higher mean log-likelihood of
 * its last E-step; this guards the chain against a pair that leaves the
 * method's basin from its first start.  Outputs (host):
 * R_rel (F-1 x 9), t_rel (F-1 x 3) with frame-k coordinates = R_rel[k]
 * (frame-(k+1) coordinates) + t_rel[k]; R_abs (F x 9), t_abs (F x 3), the
 * pose of every frame in frame 0 (frame 0 the identity), composed in FP64;
 * iters and status (nullable) per frame pair.  A singular pair keeps its last
 * good transform in the chain and, with status NULL, makes the call return
 * HGMM_ESINGULAR.  Errors: HGMM_EINVAL (F < 2, bad offsets or parameters,
 * null pointer, workspace below hgmm_odometry_workspace_bytes),
 * HGMM_ETOOFEW, HGMM_ENONFINITE, HGMM_EHIP.  Synchronises `stream`. */
size_t hgmm_odometry_workspace_bytes(const int64_t *offsets, int F, int levels);
int hgmm_odometry(const float *d_xyz, const int64_t *offsets, int F, const hgmm_build_params *bp,
                  const hgmm_reg_params *rp, const double *R0, const double *t0, int prior_restart, void *d_ws,
                  size_t ws_bytes, void *stream, hgmm_tree *forest, double *R_rel, double *t_rel, double *R_abs,
                  double *t_abs, int *iters, int *status);

/* ---- learned warm start ---------------------------------------------------
 * Not part of the paper: a small network that maps the coarse GMMs of both
 * clouds to an initial transform for hgmm_register / hgmm_register_batch.
 *
 * Features (hgmm_warm_features): for each listed tree, the 64 nodes of level 1
 * as (global weight, mean (3), upper covariance xx xy xz yy yz zz (6)) in the
 * cloud's canonical frame u = E (p - c) / s, where c is the cloud mean, s its
 * RMS radius and E the principal axes of the root covariance (rows, sign rule
 * of the node eigenvectors, last row negated if det E < 0).  Dead nodes are
 * zero.  d_feat receives n x 640 floats, d_frames n x 13 doubles (E row-major,
 * c, s); all device memory.  Synchronises `stream`.
 *
 * Network (hgmm_mlp): 1280 -> 512 -> 512 -> 512 -> 9, exact GELU after the
 * hidden layers; bf16 weights and activations into v_mfma_f32_16x16x32_bf16
 * with FP32 accumulation, FP32 biases, FP32 master weights and Adam state.
 * Input row = [source 640 | target 640] FP32 (converted to bf16 inside);
 * output row = [first two columns of Rc (6), tc (3)] where Rc, tc map target
 * canonical coordinates to source canonical coordinates.  Parameters are
 * flattened W1 b1 W2 b2 W3 b3 W4 b4 with W_l row-major [in x out]
 * (hgmm_mlp_param_count() floats).  The loss of a row against target T is
 * sum_c w_c (y_c - T_c)^2 / 2 with w = 1 on the 6D part and trans_weight on
 * the translation, averaged over rows.
 *
 * hgmm_warm_head_pose turns rows into transforms (Gram-Schmidt on the 6D
 * part, composed with the two frames): d_R0 (P x 9), d_t0 (P x 3) doubles;
 * hgmm_warm_head_target is its inverse for training targets. */
typedef struct hgmm_mlp_s *hgmm_mlp;
int64_t hgmm_mlp_param_count(void);
int hgmm_mlp_create(uint64_t seed, hgmm_mlp *out);
void hgmm_mlp_destroy(hgmm_mlp mlp);
int hgmm_mlp_get_params(hgmm_mlp mlp, float *host_params);
int hgmm_mlp_set_params(hgmm_mlp mlp, const float *host_params);
int hgmm_mlp_forward(hgmm_mlp mlp, const float *d_X, int P, float *d_Y, void *stream);
/* One Adam step (lr, beta 0.9 / 0.999, eps 1e-8) on rows d_X against d_T;
 * *loss (nullable, host) is the mean loss before the step. */
int hgmm_mlp_train_step(hgmm_mlp mlp, const float *d_X, const float *d_T, int P, float lr, float trans_weight,
                        void *stream, double *loss);
/* Forward + backward only; host_grads (nullable) receives the parameter
 * gradients in the flattened layout. */
int hgmm_mlp_backward(hgmm_mlp mlp, const float *d_X, const float *d_T, int P, float trans_weight, void *stream,
                      float *host_grads, double *loss);
int hgmm_warm_features(hgmm_tree forest, const int32_t *h_tree_ids, int n, double reg_eps, float *d_feat,
                       double *d_frames, void *stream);
int hgmm_warm_head_pose(const float *d_Y, const double *d_fr_src, const double *d_fr_tgt, int P, double *d_R0,
                        double *d_t0, void *stream);
int hgmm_warm_head_target(const double *d_R, const double *d_t, const double *d_fr_src, const double *d_fr_tgt, int P,
                          float *d_T, void *stream);
/* Warm-started registration with the plain method as the fallback and the
 * arbiter: pair b (target cloud b, CSR offsets, B pairs) onto tree b of the
 * forest, starting from R0[9 b..], t0[3 b..] (host; the head's transforms).
 * With coarse_levels > 0 and a tree deeper than that, the descent is first
 * capped at coarse_levels levels (a wider basin; a pair whose capped run
 * fails keeps R0, t0), then the registration runs over the whole tree.
 * rule 0: every pair is also registered from the identity and keeps the
 * result with the higher final log-likelihood (a failed warm run falls
 * back); rule 1: one E-step at the identity, and a pair whose final
 * log-likelihood is below the identity's (or whose warm run failed) is
 * registered again from the identity.  Outputs as hgmm_register_batch, plus
 * fallback[b] = 1 where the result is the plain method's.  The workspace is
 * hgmm_register_batch_workspace_bytes.  With reg_sort the moving points are
 * put in Morton order once, by the first of these runs, and the later runs
 * reuse that order (it depends on the points and the trees' frames, not on
 * the poses).  Synchronises `stream`. */
int hgmm_register_warm_batch(hgmm_tree forest, const float *d_xyz, const int64_t *offsets, int B,
                             const hgmm_reg_params *p, int coarse_levels, int rule, const double *R0,
                             const double *t0, void *d_ws, size_t ws_bytes, void *stream, double *R, double *t,
                             int *iters, double *loglik, int *status, int32_t *fallback);
/* C = op(A) op(B) on the MLP's bf16 MFMA GEMM (A, B raw bf16, C FP32). */
int hgmm_gemm_bf16(int ta, int tb, int M, int N, int K, const uint16_t *d_A, int lda, const uint16_t *d_B, int ldb,
                   float *d_C, int ldc, void *stream);

/* FP64 host copy of tree `index` of the forest (all arrays caller-allocated). */
int hgmm_tree_export(hgmm_tree tree, int index, hgmm_tree_host *out);
/* Per-point node labels of tree `index`: d_labels[l * n_points + i] is the
 * index inside level l of the node that point i of the model cloud belongs to
 * (-1 if its path ended above level l).  Device int32, caller-allocated. */
int hgmm_tree_labels(hgmm_tree tree, int index, int32_t *d_labels, void *stream);
/* Builds a single-tree handle from a host tree (every field is used as
 * given, origin and extent included).  Node arrays are copied; the handle has
 * no per-point labels. */
int hgmm_tree_import(const hgmm_tree_host *in, void *stream, hgmm_tree *out);
/* levels, total nodes, origin and extent of tree `index`. */
int hgmm_tree_info(hgmm_tree tree, int index, int *levels, int64_t *n_nodes, double origin[3], double *extent);
void hgmm_tree_destroy(hgmm_tree tree);

/* Launch shapes of the construction and registration kernels (process wide,
 * the search space of the autotuner).  Construction of a level: a parent with
 * at most block64_max points runs all its EM iterations in one 64-thread
 * block, at most block256_max in one 256-thread block, at most block512_max
 * in one 512-thread block; a larger parent is cut into tiles of tile_threads
 * threads and each EM iteration is one tile launch, plus one final M-step
 * launch per level.  When a level's tile launch has at most fold_tiles tiles,
 * every tile block also folds its parent's partials of the previous iteration
 * and runs that M-step (no launch between iterations); with more tiles that
 * fold runs once per parent in a launch of its own between iterations.  Points per
 * tile are level_points / target_tiles rounded up to a multiple of 64 and
 * clamped to [min_tile, max_tile].  Registration: reg_tile points per
 * 256-thread descent block (a multiple of 256); reg_chunk iterations are
 * queued between two convergence checks on the host.  reg_graph = 1 captures
 * one chunk (descent + normal equations, reg_chunk times) in a hipGraph on a
 * library-owned stream joined to the caller's by events; the instantiated
 * graph is kept in the tree handle and reused while the call's sizes,
 * buffers and knobs stay the same.  Timing with hgmm_profile(1) uses plain
 * launches.  reg_sort = 1 sorts the moving points of every pair by the Morton
 * code of their position in the model tree's frame (one radix sort per call,
 * inside the workspace) so that neighbouring lanes stop at the same nodes;
 * the results change only by summation order.
 * reg_lds_levels = 3 also stages level 2 (512 nodes, 48 KB per block), which
 * pays for large registration tiles.
 * build_graph = 1 plans every construction level on the device (the same
 * jobs, classes and tiles as the host planner) and runs all launches of a
 * construction as one hipGraph, captured on the first call of a shape (cloud
 * sizes and depths, buffers, parameters, launch shapes) and cached in the
 * handle; no host round trip between levels.  build_graph = 2 issues the
 * same device-planned launches directly on the stream, without a graph (no
 * capture, no graph launch; the host enqueues while the GPU runs).  Results
 * equal those of build_graph = 0.  Neither is used while hgmm_profile is on.
 * reg_atomics selects how the registration descent adds its moments: 0
 * (default) in fixed point (two 64-bit integer words per value), whose
 * integer sums do not depend on the order of the additions, so moments and
 * poses are bitwise reproducible from run to run; 1 as FP64 atomic adds of
 * the FP32 run sums into FP64 node bins, whose order, and so the last bits of
 * the moments, vary between runs (kept to compare against).
 * Defaults 256, 2048, 8192, 1024, 1024, 4096, 512, 4, 0, 0, 256, 2, 0, 0,
 * 1024. */
typedef struct hgmm_tuning {
  int32_t block64_max, block256_max, block512_max;
  int32_t min_tile, target_tiles, max_tile;
  int32_t reg_tile, reg_chunk;
  int32_t reg_graph;  /* 1: each chunk of registration iterations is one hipGraph launch */
  int32_t reg_sort;   /* 1: the moving cloud is put in Morton order once per registration call */
  int32_t tile_threads; /* threads per construction tile: 256, 512 or 1024 */
  int32_t reg_lds_levels; /* tree levels whose scoring records the descent stages in LDS: 2 or 3 */
  int32_t build_graph;    /* 1: construction planned on the device and run as one hipGraph; 2: the same
                             device-planned launches issued on the stream */
  int32_t reg_atomics;    /* 0: fixed-point moments (reproducible); 1: FP64 atomic moments */
  int32_t fold_tiles;     /* largest tile launch whose blocks fold the previous iteration themselves */
} hgmm_tuning;

/* Constructions of a handle so far: those planned on the device (a replay of
 * its cached construction graph with build_graph = 1, or the same launches on
 * the stream with build_graph = 2), the graphs captured, and those planned on
 * the host (build_graph = 0, the first construction of a new shape with
 * build_graph = 1 or 2, and one whose plan had work where the device-planned
 * launches had none).  Host outputs; HGMM_EINVAL on a null argument. */
int hgmm_build_graph_stats(hgmm_tree tree, int64_t *replays, int64_t *captures, int64_t *host_builds);

/* Set (after validation) or read the launch shapes.  hgmm_set_tuning returns
 * HGMM_EINVAL, changing nothing, unless 0 <= block64_max <= block256_max <=
 * block512_max <= 1<<20, 64 <= min_tile <= max_tile <= 1<<20,
 * target_tiles >= 1, 256 <= reg_tile <= 1<<20, 1 <= reg_chunk <= 64 and
 * reg_graph, reg_sort in {0, 1}, build_graph in {0, 1, 2}, tile_threads in
 * {256, 512, 1024} and reg_lds_levels in {2, 3}.
 * Values are rounded up to the multiples stated above.  Not thread-safe
 * against concurrent calls of the library. */
int hgmm_set_tuning(const hgmm_tuning *t);
int hgmm_get_tuning(hgmm_tuning *t);

/* Autotuner of the launch shapes for one workload.  Builds the forest of the
 * B source clouds (CSR: d_src SoA over src_offsets[B], levels[b] per tree,
 * parameters bp) and, when d_tgt is not NULL, registers the B target clouds
 * (tgt_offsets, parameters rp, from the identity) under candidate settings,
 * timing each run with HIP events on `stream` (best of `reps`), and moves one
 * knob at a time to the fastest of its candidates for up to `passes` sweeps.
 * On success the fastest setting is in effect and copied to *best, with its
 * time in *best_ms and the time of the starting setting in *start_ms (either
 * may be NULL).  d_ws must hold both the construction and the registration
 * workspace of this batch.  On failure the starting setting is restored.
 * The search runs the whole workload tens of times; results of the method do
 * not depend on the launch shapes beyond floating-point summation order. */
/* Workspace bytes for hgmm_autotune (tgt_offsets may be NULL: construction
 * only); 0 for invalid arguments. */
size_t hgmm_autotune_workspace_bytes(const int64_t *src_offsets, const int32_t *levels, const int64_t *tgt_offsets,
                                     int B);
int hgmm_autotune(const float *d_src, const int64_t *src_offsets, const int32_t *levels, int B,
                  const float *d_tgt, const int64_t *tgt_offsets, const hgmm_build_params *bp,
                  const hgmm_reg_params *rp, void *d_ws, size_t ws_bytes, void *stream, int reps,
                  int passes, hgmm_tuning *best, double *best_ms, double *start_ms);

/* Benchmark instrumentation.  hgmm_profile(1) brackets every kernel launch
 * of hgmm_build / hgmm_register with HIP events on the caller's stream;
 * hgmm_profile_read returns, per kernel kind, the summed event time (ms), the
 * number of timed launches and the work units they processed (points, or
 * point-iterations for the block construction kernels, or nodes for the
 * normal equations).  Every launch counts, also registration launches
 * queued after every pair had converged (they exit at once).  Kinds: 0 construction EM tile iteration,
 * 1 construction EM in one block per parent, 2 partition, 3 stable split, 4 registration
 * descent, 5 normal equations + solve, 6 root statistics, 7 construction
 * M-step of the tiled parents (units: parents), 8 single-level E-step,
 * 9 soft multi-path E-step.  Process-wide, not
 * thread-safe. */
int hgmm_profile(int enable);
void hgmm_profile_reset(void);
int hgmm_profile_read(int kind, double *total_ms, int64_t *launches, double *units);
/* For the registration descent (kind 4): the points its timed launches
 * actually processed (pairs already converged are skipped inside a launch)
 * and the tree levels those points scored, counted on the device (one
 * 64-bit atomic add per block while profiling).  Other kinds report 0. */
int hgmm_profile_work(int kind, double *points, double *levels);

/* Thread-local description of the last failure on this thread. */
const char *hgmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
