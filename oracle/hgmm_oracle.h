/*
 * FP64 single-threaded CPU oracle for GMM-Tree construction and
 * GMM-Tree registration (Eckart, Kim, Kautz, "Fast and Accurate Point Cloud
 * Registration using Trees of Gaussian Mixtures").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Conventions
 *   - Points arrive as FP32 SoA (x[n], y[n], z[n]) and are widened exactly.
 *   - Level l of a tree holds 8^(l+1) nodes; node k of level l has children
 *     8k..8k+7 at level l+1.  Level 0 nodes are the children of the root.
 *     Nodes are stored level-major; level l starts at (8^(l+1) - 8) / 7.
 *   - A covariance is packed as [xx, xy, xz, yy, yz, zz] and always includes
 *     the regularisation eps*I.
 *   - Eigenvalues are sorted lam1 >= lam2 >= lam3; eigenvector a is stored as
 *     row a of a 3x3 row-major block; its largest-|.| component is positive
 *     (lower index wins equal magnitudes).
 */
#ifndef HGMM_ORACLE_H
#define HGMM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t levels;
  int32_t pad_;
  int64_t n_nodes;
  int64_t n_points;
  double origin[3];      /* mean of the model cloud; centre of the M-step rotation increments */
  double extent;         /* bounding-box diagonal of the model cloud */
  double root_cov[6];
  double root_lam[3];
  double root_evec[9];
  int32_t *live;         /* n_nodes */
  int32_t *has_children; /* n_nodes */
  int64_t *count;        /* n_nodes: size of the node's hard partition */
  double *pi;            /* n_nodes: weight inside the sibling group */
  double *pig;           /* n_nodes: product of weights from the root */
  double *mu;            /* 3 n_nodes */
  double *cov;           /* 6 n_nodes */
  double *lam;           /* 3 n_nodes */
  double *evec;          /* 9 n_nodes */
  double *kappa;         /* n_nodes: lam3 / (lam1 + lam2 + lam3) */
} ot_tree;

enum { OT_OK = 0, OT_EINVAL = -1, OT_ETOOFEW = -2, OT_ESINGULAR = -6 };

int64_t oracle_level_offset(int level);

int oracle_eigh3(const double cov[6], double lam[3], double evec[9]);
void oracle_octant_init(const double mu[3], const double lam[3], const double evec[9], double eps,
                        double child_mu[24], double child_cov[48]);
int oracle_em_partition(const double *pts, int64_t n, int iters, double eps, double min_mass,
                        double pi[8], double mu[24], double cov[48], int32_t live[8],
                        double *resp, int32_t *label, double nk[8]);

int oracle_build_root(const float *xyz, int64_t n, double eps, ot_tree *t);
int oracle_build_level(const float *xyz, int64_t n, int level, int iters, double eps, double min_mass,
                       ot_tree *t, int32_t *labels);
int oracle_build(const float *xyz, int64_t n, int levels, int iters, double eps, double min_mass,
                 ot_tree *t, int32_t *labels);

int oracle_estep(const ot_tree *t, const float *xyz, int64_t n, const double R[9], const double tv[3],
                 double lambda_c, int32_t *stop_node, int32_t *stop_level, double *gamma,
                 double *min_gap, double *bins, double *loglik);
int oracle_normal_equations(const ot_tree *t, const double *bins, int64_t n, double H[36], double g[6]);
int oracle_solve_update(const double H[36], const double g[6], const double origin[3], double R[9],
                        double tv[3], double x[6]);
int oracle_register(const ot_tree *t, const float *xyz, int64_t n, int max_iters, double lambda_c,
                    double tol_rot, double tol_trans, double R[9], double tv[3], int *iters,
                    double *loglik, double *trace);
/* Single-level variant ("GMM J=n"): the live nodes of tree level `level`
 * (J = 8^(level+1)) as one mixture with their global weights; every point is
 * scored against every component.  Outputs as oracle_estep (stop_node: the
 * chosen component, -1 when the level has no live node). */
int oracle_estep_flat(const ot_tree *t, int level, const float *xyz, int64_t n, const double R[9],
                      const double tv[3], int32_t *stop_node, double *gamma, double *min_gap, double *bins,
                      double *loglik);
int oracle_register_flat(const ot_tree *t, int level, const float *xyz, int64_t n, int max_iters, double tol_rot,
                         double tol_trans, double R[9], double tv[3], int *iters, double *loglik);
/* Soft multi-path E-step: every branch whose path expectation (the product of
 * sibling posteriors from the root) is at least tau, stop nodes weighted by
 * it; bins {E, E q (3), E, E d_M^2}; margin: per point the smallest
 * |E - tau| / tau compared; stops: per point the number of nodes reached. */
int oracle_estep_soft(const ot_tree *t, const float *xyz, int64_t n, const double R[9], const double tv[3],
                      double lambda_c, double tau, double *bins, double *loglik, double *margin, int32_t *stops);
int oracle_register_soft(const ot_tree *t, const float *xyz, int64_t n, double lambda_c, double tau, int max_iters,
                         double tol_rot, double tol_trans, double R[9], double tv[3], int *iters, double *loglik);

#ifdef __cplusplus
}
#endif
#endif
