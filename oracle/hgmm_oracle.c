/*
 * FP64 single-threaded CPU oracle (TEST INFRASTRUCTURE ONLY; see hgmm_oracle.h).
 *
 * What each function follows in the paper (Eckart, Kim, Kautz, 2018):
 *   - mixture density and responsibilities ................ Sec. 3, Eq. 2-3
 *   - tree of 8-component mixtures, one child mixture per
 *     component, built top-down ............................ Sec. 3 end, Sec. 4.1
 *     (the construction itself is delegated by the paper to
 *     Eckart et al. CVPR 2016; the steps below are this
 *     project's reading: PCA-octant initialisation, a fixed
 *     number of EM iterations per parent, hard partition by
 *     the most likely child, regularisation eps*I, children
 *     whose soft mass drops below min_mass die)
 *   - max-likelihood descent with the complexity stop ...... Sec. 4.1, Algorithm 1
 *   - moments of the selected node ........................ Algorithm 1, Eq. 9
 *   - cluster-reduced criterion in PCA form ............... Sec. 4.2, Eq. 8-11
 *   - weighted point-to-plane least squares with a
 *     small-angle linearisation ........................... Sec. 4.2, appendix Eq. 12-16
 *   - the single-level variant "GMM J=n" (every component
 *     scored for every point, no tree descent) ............ Sec. 5, list of variants
 *   - the soft multi-path E-step: every branch whose path
 *     expectation stays above a threshold, weighted by it . Sec. 4.1 (logarithmic search)
 * Plain loops, no blocking, no SIMD, libm only.
 */
#include "hgmm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define LOG_2PI 1.8378770664093453

int64_t oracle_level_offset(int level) {
  int64_t off = 0, w = 8;
  for (int l = 0; l < level; ++l) {
    off += w;
    w *= 8;
  }
  return off;
}

/* ------------------------------------------------------------------------ */
/* 3x3 symmetric eigen-decomposition by cyclic Jacobi rotations              */
/* ------------------------------------------------------------------------ */

static void unpack_sym(const double c[6], double a[3][3]) {
  a[0][0] = c[0]; a[0][1] = c[1]; a[0][2] = c[2];
  a[1][0] = c[1]; a[1][1] = c[3]; a[1][2] = c[4];
  a[2][0] = c[2]; a[2][1] = c[4]; a[2][2] = c[5];
}

int oracle_eigh3(const double cov[6], double lam[3], double evec[9]) {
  double a[3][3], v[3][3];
  unpack_sym(cov, a);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    double diag = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]);
    if (off <= 1e-300 || off <= 1e-20 * diag) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        /* rotation angle that zeroes a[p][q]: tan(2 phi) = 2 a_pq / (a_qq - a_pp) */
        double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0);
        double s = t * c;
        /* A <- J^T A J with J the Givens rotation in the (p, q) plane */
        for (int k = 0; k < 3; ++k) {
          double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - s * vkq;
          v[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
  /* columns of v are eigenvectors; sort by eigenvalue, descending */
  int idx[3] = {0, 1, 2};
  double d[3] = {a[0][0], a[1][1], a[2][2]};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (d[idx[j]] > d[idx[i]]) {
        int tmp = idx[i];
        idx[i] = idx[j];
        idx[j] = tmp;
      }
  for (int r = 0; r < 3; ++r) {
    int col = idx[r];
    lam[r] = d[col];
    double e[3] = {v[0][col], v[1][col], v[2][col]};
    int big = 0;
    for (int k = 1; k < 3; ++k)
      if (fabs(e[k]) > fabs(e[big])) big = k;
    double sg = e[big] < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 3; ++k) evec[3 * r + k] = sg * e[k];
  }
  return OT_OK;
}

/* ------------------------------------------------------------------------ */
/* PCA-octant initialisation of the 8 children of a Gaussian                */
/* ------------------------------------------------------------------------ */

/* Child k covers the octant of the parent's eigenbasis with sign s_a = +1 when
 * bit a of k is 0 and -1 otherwise.  Along each eigen-axis the restricted
 * Gaussian is a half-normal of scale sqrt(lam_a): mean sqrt(2/pi) sqrt(lam_a),
 * variance (1 - 2/pi) lam_a, and the three axes stay independent. */
void oracle_octant_init(const double mu[3], const double lam[3], const double evec[9], double eps,
                        double child_mu[24], double child_cov[48]) {
  const double pi = 3.14159265358979323846;
  double lr[3];
  for (int a = 0; a < 3; ++a) {
    lr[a] = lam[a] - eps;
    if (lr[a] < 0.0) lr[a] = 0.0;
  }
  for (int k = 0; k < 8; ++k) {
    for (int i = 0; i < 3; ++i) {
      double m = mu[i];
      for (int a = 0; a < 3; ++a) {
        double s = ((k >> a) & 1) ? -1.0 : 1.0;
        m += s * sqrt(2.0 / pi) * sqrt(lr[a]) * evec[3 * a + i];
      }
      child_mu[3 * k + i] = m;
    }
    double c[3][3] = {{0}};
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[i][j] += (1.0 - 2.0 / pi) * lr[a] * evec[3 * a + i] * evec[3 * a + j];
    double *o = child_cov + 6 * k;
    o[0] = c[0][0] + eps; o[1] = c[0][1]; o[2] = c[0][2];
    o[3] = c[1][1] + eps; o[4] = c[1][2]; o[5] = c[2][2] + eps;
  }
}

/* ------------------------------------------------------------------------ */
/* Gaussian log-score via Cholesky                                          */
/* ------------------------------------------------------------------------ */

/* lower Cholesky factor of a packed SPD covariance; returns 0 on failure */
static int chol3(const double c[6], double L[3][3]) {
  double a[3][3];
  unpack_sym(c, a);
  memset(L, 0, sizeof(double) * 9);
  for (int j = 0; j < 3; ++j) {
    double s = a[j][j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(s > 0.0)) return 0;
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < 3; ++i) {
      double t = a[i][j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  return 1;
}

/* squared Mahalanobis distance of d under L L^T */
static double maha2(const double L[3][3], const double d[3]) {
  double w0 = d[0] / L[0][0];
  double w1 = (d[1] - L[1][0] * w0) / L[1][1];
  double w2 = (d[2] - L[2][0] * w0 - L[2][1] * w1) / L[2][2];
  return w0 * w0 + w1 * w1 + w2 * w2;
}

static double logdet_from_chol(const double L[3][3]) {
  return 2.0 * (log(L[0][0]) + log(L[1][1]) + log(L[2][2]));
}

/* ------------------------------------------------------------------------ */
/* EM of one 8-component mixture on one parent's partition                  */
/* ------------------------------------------------------------------------ */

int oracle_em_partition(const double *pts, int64_t n, int iters, double eps, double min_mass,
                        double pi[8], double mu[24], double cov[48], int32_t live[8],
                        double *resp, int32_t *label, double nk_out[8]) {
  double *r = resp ? resp : (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 8);
  double L[8][3][3], logdet[8];
  double nk[8] = {0};
  for (int it = 0; it < iters; ++it) {
    /* E-step (Eq. 3): responsibilities over the live children */
    for (int k = 0; k < 8; ++k)
      if (live[k]) {
        if (!chol3(cov + 6 * k, L[k])) { if (!resp) free(r); return OT_ESINGULAR; }
        logdet[k] = logdet_from_chol(L[k]);
      }
    for (int64_t i = 0; i < n; ++i) {
      double s[8], smax = -INFINITY;
      for (int k = 0; k < 8; ++k) {
        if (!live[k]) { s[k] = -INFINITY; continue; }
        double d[3] = {pts[3 * i] - mu[3 * k], pts[3 * i + 1] - mu[3 * k + 1], pts[3 * i + 2] - mu[3 * k + 2]};
        s[k] = log(pi[k]) - 0.5 * logdet[k] - 0.5 * maha2(L[k], d);
        if (s[k] > smax) smax = s[k];
      }
      double den = 0.0;
      for (int k = 0; k < 8; ++k) den += live[k] ? exp(s[k] - smax) : 0.0;
      for (int k = 0; k < 8; ++k) r[8 * i + k] = live[k] ? exp(s[k] - smax) / den : 0.0;
    }
    /* M-step: soft counts, dead rule, means, then covariances about the new means */
    double total = 0.0;
    for (int k = 0; k < 8; ++k) {
      nk[k] = 0.0;
      if (!live[k]) continue;
      for (int64_t i = 0; i < n; ++i) nk[k] += r[8 * i + k];
      if (nk[k] < min_mass) live[k] = 0;
      else total += nk[k];
    }
    for (int k = 0; k < 8; ++k) {
      if (!live[k]) { pi[k] = 0.0; continue; }
      double m[3] = {0, 0, 0};
      for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) m[c] += r[8 * i + k] * pts[3 * i + c];
      for (int c = 0; c < 3; ++c) mu[3 * k + c] = m[c] / nk[k];
      double s6[6] = {0, 0, 0, 0, 0, 0};
      for (int64_t i = 0; i < n; ++i) {
        double d[3] = {pts[3 * i] - mu[3 * k], pts[3 * i + 1] - mu[3 * k + 1], pts[3 * i + 2] - mu[3 * k + 2]};
        double w = r[8 * i + k];
        s6[0] += w * d[0] * d[0]; s6[1] += w * d[0] * d[1]; s6[2] += w * d[0] * d[2];
        s6[3] += w * d[1] * d[1]; s6[4] += w * d[1] * d[2]; s6[5] += w * d[2] * d[2];
      }
      for (int c = 0; c < 6; ++c) cov[6 * k + c] = s6[c] / nk[k];
      cov[6 * k + 0] += eps; cov[6 * k + 3] += eps; cov[6 * k + 5] += eps;
      pi[k] = nk[k] / total;
    }
  }
  if (nk_out) memcpy(nk_out, nk, sizeof(nk));
  /* hard partition with the final parameters: most likely live child, lowest index on ties */
  if (label) {
    int any = 0;
    for (int k = 0; k < 8; ++k)
      if (live[k]) {
        any = 1;
        if (!chol3(cov + 6 * k, L[k])) { if (!resp) free(r); return OT_ESINGULAR; }
        logdet[k] = logdet_from_chol(L[k]);
      }
    for (int64_t i = 0; i < n; ++i) {
      int best = -1;
      double bs = -INFINITY;
      if (any)
        for (int k = 0; k < 8; ++k) {
          if (!live[k]) continue;
          double d[3] = {pts[3 * i] - mu[3 * k], pts[3 * i + 1] - mu[3 * k + 1], pts[3 * i + 2] - mu[3 * k + 2]};
          double s = log(pi[k]) - 0.5 * logdet[k] - 0.5 * maha2(L[k], d);
          if (best < 0 || s > bs) { bs = s; best = k; }
        }
      label[i] = best;
    }
  }
  if (!resp) free(r);
  return OT_OK;
}

/* ------------------------------------------------------------------------ */
/* Tree construction                                                         */
/* ------------------------------------------------------------------------ */

int oracle_build_root(const float *xyz, int64_t n, double eps, ot_tree *t) {
  if (n < 8) return OT_ETOOFEW;
  const float *x = xyz, *y = xyz + n, *z = xyz + 2 * n;
  double m[3] = {0, 0, 0}, lo[3], hi[3];
  for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    for (int c = 0; c < 3; ++c) {
      if (!isfinite(p[c])) return OT_EINVAL;
      m[c] += p[c];
      if (p[c] < lo[c]) lo[c] = p[c];
      if (p[c] > hi[c]) hi[c] = p[c];
    }
  }
  for (int c = 0; c < 3; ++c) m[c] /= (double)n;
  double s6[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    double d[3] = {x[i] - m[0], y[i] - m[1], z[i] - m[2]};
    s6[0] += d[0] * d[0]; s6[1] += d[0] * d[1]; s6[2] += d[0] * d[2];
    s6[3] += d[1] * d[1]; s6[4] += d[1] * d[2]; s6[5] += d[2] * d[2];
  }
  for (int c = 0; c < 6; ++c) t->root_cov[c] = s6[c] / (double)n;
  t->root_cov[0] += eps; t->root_cov[3] += eps; t->root_cov[5] += eps;
  oracle_eigh3(t->root_cov, t->root_lam, t->root_evec);
  for (int c = 0; c < 3; ++c) t->origin[c] = m[c];
  t->extent = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                   (hi[2] - lo[2]) * (hi[2] - lo[2]));
  t->n_points = n;
  return OT_OK;
}

/* Builds level `level` from the parents at level-1 (the root for level 0).
 * labels is level-major [levels][n]: row level-1 is read (ignored at level 0),
 * row `level` is written (-1 for points whose parent is a leaf). */
int oracle_build_level(const float *xyz, int64_t n, int level, int iters, double eps, double min_mass,
                       ot_tree *t, int32_t *labels) {
  const float *x = xyz, *y = xyz + n, *z = xyz + 2 * n;
  int64_t nparents = 1;
  for (int l = 0; l < level; ++l) nparents *= 8;
  int64_t off = oracle_level_offset(level);
  int64_t poff = level > 0 ? oracle_level_offset(level - 1) : 0;
  int32_t *out = labels + (int64_t)level * n;
  const int32_t *in = level > 0 ? labels + (int64_t)(level - 1) * n : NULL;
  for (int64_t i = 0; i < n; ++i) out[i] = -1;
  for (int64_t k = 0; k < 8 * nparents; ++k) {
    int64_t g = off + k;
    t->live[g] = 0; t->has_children[g] = 0; t->count[g] = 0;
    t->pi[g] = 0.0; t->pig[g] = 0.0; t->kappa[g] = 0.0;
    for (int c = 0; c < 3; ++c) { t->mu[3 * g + c] = 0.0; t->lam[3 * g + c] = 0.0; }
    for (int c = 0; c < 6; ++c) t->cov[6 * g + c] = 0.0;
    for (int c = 0; c < 9; ++c) t->evec[9 * g + c] = 0.0;
  }
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)n);
  int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int status = OT_OK;
  for (int64_t p = 0; p < nparents && status == OT_OK; ++p) {
    const double *pmu, *plam, *pevec;
    double pig_parent;
    if (level == 0) {
      pmu = t->origin; plam = t->root_lam; pevec = t->root_evec; pig_parent = 1.0;
    } else {
      int64_t pg = poff + p;
      t->has_children[pg] = 0;
      if (!t->live[pg]) continue;
      pmu = t->mu + 3 * pg; plam = t->lam + 3 * pg; pevec = t->evec + 9 * pg; pig_parent = t->pig[pg];
    }
    /* the parent's partition, in point-index order */
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
      if (level == 0 || in[i] == (int32_t)p) {
        idx[m] = i;
        pts[3 * m] = x[i]; pts[3 * m + 1] = y[i]; pts[3 * m + 2] = z[i];
        ++m;
      }
    if (m == 0) continue; /* an empty partition leaves the parent a leaf */
    double cpi[8], cmu[24], ccov[48];
    int32_t clive[8];
    oracle_octant_init(pmu, plam, pevec, eps, cmu, ccov);
    for (int k = 0; k < 8; ++k) { cpi[k] = 0.125; clive[k] = 1; }
    status = oracle_em_partition(pts, m, iters, eps, min_mass, cpi, cmu, ccov, clive, NULL, lab, NULL);
    if (status != OT_OK) break;
    int any = 0;
    for (int k = 0; k < 8; ++k) {
      int64_t g = off + 8 * p + k;
      if (!clive[k]) continue;
      any = 1;
      t->live[g] = 1;
      t->pi[g] = cpi[k];
      t->pig[g] = cpi[k] * pig_parent;
      for (int c = 0; c < 3; ++c) t->mu[3 * g + c] = cmu[3 * k + c];
      for (int c = 0; c < 6; ++c) t->cov[6 * g + c] = ccov[6 * k + c];
      oracle_eigh3(t->cov + 6 * g, t->lam + 3 * g, t->evec + 9 * g);
      t->kappa[g] = t->lam[3 * g + 2] / (t->lam[3 * g] + t->lam[3 * g + 1] + t->lam[3 * g + 2]);
    }
    if (level > 0) t->has_children[poff + p] = any;
    for (int64_t j = 0; j < m; ++j)
      if (lab[j] >= 0) {
        int64_t child = 8 * p + lab[j];
        out[idx[j]] = (int32_t)child;
        t->count[off + child] += 1;
      }
  }
  free(idx);
  free(pts);
  free(lab);
  return status;
}

int oracle_build(const float *xyz, int64_t n, int levels, int iters, double eps, double min_mass,
                 ot_tree *t, int32_t *labels) {
  if (levels < 1 || levels > 6 || iters < 0) return OT_EINVAL;
  t->levels = levels;
  t->n_nodes = oracle_level_offset(levels);
  int st = oracle_build_root(xyz, n, eps, t);
  if (st != OT_OK) return st;
  for (int l = 0; l < levels; ++l) {
    st = oracle_build_level(xyz, n, l, iters, eps, min_mass, t, labels);
    if (st != OT_OK) return st;
  }
  return OT_OK;
}

/* ------------------------------------------------------------------------ */
/* Registration E-step: adaptive descent and moments (Algorithm 1)           */
/* ------------------------------------------------------------------------ */

int oracle_estep(const ot_tree *t, const float *xyz, int64_t n, const double R[9], const double tv[3],
                 double lambda_c, int32_t *stop_node, int32_t *stop_level, double *gamma,
                 double *min_gap, double *bins, double *loglik) {
  const float *x = xyz, *y = xyz + n, *z = xyz + 2 * n;
  const int L = t->levels;
  double *Lc = (double *)malloc(sizeof(double) * 9 * (size_t)t->n_nodes);
  double *ld = (double *)malloc(sizeof(double) * (size_t)t->n_nodes);
  for (int64_t g = 0; g < t->n_nodes; ++g) {
    if (!t->live[g]) continue;
    double Lm[3][3];
    if (!chol3(t->cov + 6 * g, Lm)) { free(Lc); free(ld); return OT_ESINGULAR; }
    memcpy(Lc + 9 * g, Lm, sizeof(Lm));
    ld[g] = logdet_from_chol(Lm);
  }
  if (bins) memset(bins, 0, sizeof(double) * 6 * (size_t)t->n_nodes);
  double ll = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    double q[3];
    for (int r = 0; r < 3; ++r) q[r] = R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2] + tv[r];
    int64_t parent = -1;
    int64_t chosen = -1;
    int lev = 0;
    double s_best = 0.0, s_all[8], gapmin = INFINITY;
    int live_ch[8];
    for (int l = 0; l < L; ++l) {
      int64_t base = oracle_level_offset(l) + (parent < 0 ? 0 : 8 * parent);
      int kbest = -1;
      double sb = -INFINITY, s2 = -INFINITY;
      for (int k = 0; k < 8; ++k) {
        int64_t g = base + k;
        live_ch[k] = t->live[g];
        if (!live_ch[k]) { s_all[k] = -INFINITY; continue; }
        double d[3] = {q[0] - t->mu[3 * g], q[1] - t->mu[3 * g + 1], q[2] - t->mu[3 * g + 2]};
        double Lm[3][3];
        memcpy(Lm, Lc + 9 * g, sizeof(Lm));
        /* gamma[j] proportional to pi_j N(z | Theta_j), pi_j taken inside the sibling group */
        s_all[k] = log(t->pi[g]) - 0.5 * ld[g] - 0.5 * maha2(Lm, d);
        if (kbest < 0 || s_all[k] > sb) { s2 = sb; sb = s_all[k]; kbest = k; }
        else if (s_all[k] > s2) s2 = s_all[k];
      }
      if (kbest < 0) break; /* cannot happen for a live parent with live children */
      if (s2 > -INFINITY && sb - s2 < gapmin) gapmin = sb - s2;
      chosen = base + kbest;
      s_best = sb;
      lev = l;
      int stop = (t->kappa[chosen] <= lambda_c) || (l == L - 1) || !t->has_children[chosen];
      if (stop) break;
      parent = chosen - oracle_level_offset(l);
    }
    double den = 0.0;
    for (int k = 0; k < 8; ++k)
      if (live_ch[k]) den += exp(s_all[k] - s_best);
    double gm = 1.0 / den;
    int64_t g = chosen;
    double d[3] = {q[0] - t->mu[3 * g], q[1] - t->mu[3 * g + 1], q[2] - t->mu[3 * g + 2]};
    double Lm[3][3];
    memcpy(Lm, Lc + 9 * g, sizeof(Lm));
    double m2 = maha2(Lm, d);
    if (stop_node) stop_node[i] = (int32_t)g;
    if (stop_level) stop_level[i] = lev;
    if (gamma) gamma[i] = gm;
    if (min_gap) min_gap[i] = gapmin;
    if (bins) {
      double *b = bins + 6 * g;
      b[0] += gm;
      b[1] += gm * q[0];
      b[2] += gm * q[1];
      b[3] += gm * q[2];
      b[4] += 1.0;
      b[5] += m2;
    }
    ll += log(t->pig[g]) - 0.5 * ld[g] - 0.5 * m2 - 1.5 * LOG_2PI;
  }
  if (loglik) *loglik = ll / (double)n;
  free(Lc);
  free(ld);
  return OT_OK;
}

/* ------------------------------------------------------------------------ */
/* M-step: PCA-form normal equations (Eq. 11-16)                            */
/* ------------------------------------------------------------------------ */

/* For every node j with M0_j > 0: pi*_j = M0_j / N, mu*_j = M1_j / M0_j.  Each of
 * the three eigen-directions n_l contributes one weighted point-to-plane row
 * a = [(mu*_j - o) x n_l ; n_l], weight pi*_j / lam_l, residual n_l.(mu*_j - mu_j).
 * The increment x = (omega, tau) of T(p) = p + omega x (p - o) + tau minimises
 * sum w (a.x + r)^2, i.e. H x = g with H = sum w a a^T and g = -sum w a r. */
int oracle_normal_equations(const ot_tree *t, const double *bins, int64_t n, double H[36], double g[6]) {
  memset(H, 0, sizeof(double) * 36);
  memset(g, 0, sizeof(double) * 6);
  for (int64_t j = 0; j < t->n_nodes; ++j) {
    const double *b = bins + 6 * j;
    if (!(b[0] > 0.0)) continue;
    double pis = b[0] / (double)n;
    double ms[3] = {b[1] / b[0], b[2] / b[0], b[3] / b[0]};
    double c[3] = {ms[0] - t->origin[0], ms[1] - t->origin[1], ms[2] - t->origin[2]};
    for (int l = 0; l < 3; ++l) {
      const double *nv = t->evec + 9 * j + 3 * l;
      double w = pis / t->lam[3 * j + l];
      double a[6] = {c[1] * nv[2] - c[2] * nv[1], c[2] * nv[0] - c[0] * nv[2], c[0] * nv[1] - c[1] * nv[0],
                     nv[0], nv[1], nv[2]};
      double r = nv[0] * (ms[0] - t->mu[3 * j]) + nv[1] * (ms[1] - t->mu[3 * j + 1]) + nv[2] * (ms[2] - t->mu[3 * j + 2]);
      for (int u = 0; u < 6; ++u) {
        g[u] -= w * a[u] * r;
        for (int v = 0; v < 6; ++v) H[6 * u + v] += w * a[u] * a[v];
      }
    }
  }
  return OT_OK;
}

static int chol6_solve(const double H[36], double shift, const double g[6], double x[6]) {
  double L[6][6];
  memset(L, 0, sizeof(L));
  for (int j = 0; j < 6; ++j) {
    double s = H[6 * j + j] + shift;
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(s > 0.0)) return 0;
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < 6; ++i) {
      double t = H[6 * i + j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  double yv[6];
  for (int i = 0; i < 6; ++i) {
    double s = g[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * yv[k];
    yv[i] = s / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = yv[i];
    for (int k = i + 1; k < 6; ++k) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
  return 1;
}

int oracle_solve_update(const double H[36], const double g[6], const double origin[3], double R[9],
                        double tv[3], double x[6]) {
  if (!chol6_solve(H, 0.0, g, x)) {
    double tr = 0.0;
    for (int i = 0; i < 6; ++i) tr += H[7 * i];
    if (!(tr > 0.0) || !chol6_solve(H, 1e-12 * tr, g, x)) return OT_ESINGULAR;
  }
  /* exact rotation for the linearised angle vector omega (Rodrigues) */
  double w[3] = {x[0], x[1], x[2]};
  double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
  double K2[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
  double a, b;
  if (th < 1e-12) { a = 1.0; b = 0.0; }
  else { a = sin(th) / th; b = (1.0 - cos(th)) / (th * th); }
  double Ri[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ri[i][j] = (i == j ? 1.0 : 0.0) + a * K[i][j] + b * K2[i][j];
  /* T_new(p) = Ri (T(p) - o) + o + tau */
  double Rn[9], tn[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) Rn[3 * i + j] = Ri[i][0] * R[j] + Ri[i][1] * R[3 + j] + Ri[i][2] * R[6 + j];
    tn[i] = Ri[i][0] * (tv[0] - origin[0]) + Ri[i][1] * (tv[1] - origin[1]) + Ri[i][2] * (tv[2] - origin[2]) +
            origin[i] + x[3 + i];
  }
  memcpy(R, Rn, sizeof(Rn));
  memcpy(tv, tn, sizeof(tn));
  return OT_OK;
}

/* trace (nullable): per iteration 20 doubles: loglik, omega[3], tau[3], R[9], t[3], status */
int oracle_register(const ot_tree *t, const float *xyz, int64_t n, int max_iters, double lambda_c,
                    double tol_rot, double tol_trans, double R[9], double tv[3], int *iters,
                    double *loglik, double *trace) {
  if (n < 1 || max_iters < 1) return OT_EINVAL;
  double *bins = (double *)malloc(sizeof(double) * 6 * (size_t)t->n_nodes);
  int st = OT_OK, it;
  double ll = 0.0;
  *iters = 0;
  for (it = 1; it <= max_iters; ++it) {
    st = oracle_estep(t, xyz, n, R, tv, lambda_c, NULL, NULL, NULL, NULL, bins, &ll);
    if (st != OT_OK) break;
    double H[36], g[6], x[6] = {0, 0, 0, 0, 0, 0};
    oracle_normal_equations(t, bins, n, H, g);
    *iters = it;
    st = oracle_solve_update(H, g, t->origin, R, tv, x);
    if (trace) {
      double *tr = trace + 20 * (it - 1);
      tr[0] = ll;
      for (int k = 0; k < 6; ++k) tr[1 + k] = x[k];
      for (int k = 0; k < 9; ++k) tr[7 + k] = R[k];
      for (int k = 0; k < 3; ++k) tr[16 + k] = tv[k];
      tr[19] = st;
    }
    if (st != OT_OK) break;
    double wn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double tn = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
    if (wn < tol_rot && tn < tol_trans) break;
  }
  if (loglik) *loglik = ll;
  free(bins);
  return st;
}

/* Single-level variant ("GMM J=n", Sec. 5 list of variants): the live nodes of
 * one tree level form a mixture of J = 8^(level+1) components with their
 * global weights pi^g.  Every point is scored against every component (Eq. 2-3
 * with pi^g), associated with the most likely one (lowest index on exact
 * ties) and weighted by its posterior among all of them; the moments of
 * Algorithm 1 go to that component.  Renormalising the weights over the level
 * would cancel in the argmax and the posterior; the log-likelihood uses pi^g
 * as the tree's E-step does.  min_gap: top-2 score gap (natural log units). */
int oracle_estep_flat(const ot_tree *t, int level, const float *xyz, int64_t n, const double R[9],
                      const double tv[3], int32_t *stop_node, double *gamma, double *min_gap, double *bins,
                      double *loglik) {
  if (level < 0 || level >= t->levels) return OT_EINVAL;
  const float *x = xyz, *y = xyz + n, *z = xyz + 2 * n;
  const int64_t g0 = oracle_level_offset(level), J = oracle_level_offset(level + 1) - g0;
  double *Lc = (double *)malloc(sizeof(double) * 9 * (size_t)J);
  double *cst = (double *)malloc(sizeof(double) * (size_t)J);
  double *ld = (double *)malloc(sizeof(double) * (size_t)J);
  for (int64_t j = 0; j < J; ++j) {
    const int64_t g = g0 + j;
    if (!t->live[g]) continue;
    double Lm[3][3];
    if (!chol3(t->cov + 6 * g, Lm)) { free(Lc); free(cst); free(ld); return OT_ESINGULAR; }
    memcpy(Lc + 9 * j, Lm, sizeof(Lm));
    ld[j] = logdet_from_chol(Lm);
    cst[j] = log(t->pig[g]) - 0.5 * ld[j];
  }
  if (bins) memset(bins, 0, sizeof(double) * 6 * (size_t)t->n_nodes);
  double ll = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    double q[3];
    for (int r = 0; r < 3; ++r) q[r] = R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2] + tv[r];
    int64_t kb = -1;
    double sb = -INFINITY, s2 = -INFINITY;
    for (int64_t j = 0; j < J; ++j) {
      const int64_t g = g0 + j;
      if (!t->live[g]) continue;
      double d[3] = {q[0] - t->mu[3 * g], q[1] - t->mu[3 * g + 1], q[2] - t->mu[3 * g + 2]};
      double Lm[3][3];
      memcpy(Lm, Lc + 9 * j, sizeof(Lm));
      const double sj = cst[j] - 0.5 * maha2(Lm, d);
      if (kb < 0 || sj > sb) { s2 = sb; sb = sj; kb = j; }
      else if (sj > s2) s2 = sj;
    }
    if (kb < 0) {  /* no live component at this level */
      if (stop_node) stop_node[i] = -1;
      if (gamma) gamma[i] = 0.0;
      if (min_gap) min_gap[i] = INFINITY;
      continue;
    }
    /* posterior of the chosen component: 1 / sum_j exp(s_j - s_best) */
    double den = 0.0;
    for (int64_t j = 0; j < J; ++j) {
      const int64_t g = g0 + j;
      if (!t->live[g]) continue;
      double d[3] = {q[0] - t->mu[3 * g], q[1] - t->mu[3 * g + 1], q[2] - t->mu[3 * g + 2]};
      double Lm[3][3];
      memcpy(Lm, Lc + 9 * j, sizeof(Lm));
      den += exp(cst[j] - 0.5 * maha2(Lm, d) - sb);
    }
    const double gm = 1.0 / den;
    const int64_t g = g0 + kb;
    double d[3] = {q[0] - t->mu[3 * g], q[1] - t->mu[3 * g + 1], q[2] - t->mu[3 * g + 2]};
    double Lm[3][3];
    memcpy(Lm, Lc + 9 * kb, sizeof(Lm));
    const double m2 = maha2(Lm, d);
    if (stop_node) stop_node[i] = (int32_t)g;
    if (gamma) gamma[i] = gm;
    if (min_gap) min_gap[i] = (s2 > -INFINITY) ? sb - s2 : INFINITY;
    if (bins) {
      double *b = bins + 6 * g;
      b[0] += gm;
      b[1] += gm * q[0];
      b[2] += gm * q[1];
      b[3] += gm * q[2];
      b[4] += 1.0;
      b[5] += m2;
    }
    ll += log(t->pig[g]) - 0.5 * ld[kb] - 0.5 * m2 - 1.5 * LOG_2PI;
  }
  if (loglik) *loglik = ll / (double)n;
  free(Lc);
  free(cst);
  free(ld);
  return OT_OK;
}

/* Registration with the single-level variant: the EM loop of oracle_register
 * with oracle_estep_flat as the E-step. */
int oracle_register_flat(const ot_tree *t, int level, const float *xyz, int64_t n, int max_iters, double tol_rot,
                         double tol_trans, double R[9], double tv[3], int *iters, double *loglik) {
  if (n < 1 || max_iters < 1) return OT_EINVAL;
  double *bins = (double *)malloc(sizeof(double) * 6 * (size_t)t->n_nodes);
  int st = OT_OK, it;
  double ll = 0.0;
  *iters = 0;
  for (it = 1; it <= max_iters; ++it) {
    st = oracle_estep_flat(t, level, xyz, n, R, tv, NULL, NULL, NULL, bins, &ll);
    if (st != OT_OK) break;
    double H[36], g[6], x[6] = {0, 0, 0, 0, 0, 0};
    oracle_normal_equations(t, bins, n, H, g);
    *iters = it;
    st = oracle_solve_update(H, g, t->origin, R, tv, x);
    if (st != OT_OK) break;
    double wn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double tn = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
    if (wn < tol_rot && tn < tol_trans) break;
  }
  if (loglik) *loglik = ll;
  free(bins);
  return st;
}

/* Soft multi-path E-step (Sec. 4.1, logarithmic search): a point's expectation
 * of a node is the product of its posteriors among the siblings along the path
 * from the root (the expectation of a parent is the sum of its children's).
 * Every branch whose expectation is at least tau is followed; a branch below
 * tau is pruned with its subtree.  A followed node stops (by the rule of
 * Algorithm 1: complexity <= lambda_c, no live children, or the last level)
 * and receives the point with weight E, its path expectation:
 * bins[g] += {E, E q (3), E, E d_M^2}; the log-likelihood is the E-weighted
 * log density, sum_i sum_stops E (log pi^g - log|cov|/2 - d_M^2/2) / n - 3/2 log 2 pi.
 * margin (nullable): per point, the smallest |E - tau| / tau over every
 * expectation compared with tau (a pruning decision that rounding could flip).
 * stops (nullable): per point, the number of nodes it reached. */
int oracle_estep_soft(const ot_tree *t, const float *xyz, int64_t n, const double R[9], const double tv[3],
                      double lambda_c, double tau, double *bins, double *loglik, double *margin, int32_t *stops) {
  const float *x = xyz, *y = xyz + n, *z = xyz + 2 * n;
  const int L = t->levels;
  double *Lc = (double *)malloc(sizeof(double) * 9 * (size_t)t->n_nodes);
  double *ld = (double *)malloc(sizeof(double) * (size_t)t->n_nodes);
  for (int64_t g = 0; g < t->n_nodes; ++g) {
    if (!t->live[g]) continue;
    double Lm[3][3];
    if (!chol3(t->cov + 6 * g, Lm)) { free(Lc); free(ld); return OT_ESINGULAR; }
    memcpy(Lc + 9 * g, Lm, sizeof(Lm));
    ld[g] = logdet_from_chol(Lm);
  }
  if (bins) memset(bins, 0, sizeof(double) * 6 * (size_t)t->n_nodes);
  const int cap = 8 * L + 8;
  int64_t *st_g = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
  int *st_l = (int *)malloc(sizeof(int) * (size_t)cap);
  double *st_e = (double *)malloc(sizeof(double) * (size_t)cap);
  double ll = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {x[i], y[i], z[i]};
    double q[3];
    for (int r = 0; r < 3; ++r) q[r] = R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2] + tv[r];
    double mg = INFINITY;
    int ns = 0, top = 0;
    /* a virtual parent of the level-0 nodes with expectation 1 */
    int64_t parent = -1;
    int plev = -1;
    double pe = 1.0;
    for (;;) {
      /* expand `parent`: posteriors of its live children, children above tau pushed */
      const int cl = plev + 1;
      const int64_t base = oracle_level_offset(cl) + (parent < 0 ? 0 : 8 * (parent - oracle_level_offset(plev)));
      double s[8], smax = -INFINITY;
      for (int k = 0; k < 8; ++k) {
        const int64_t g = base + k;
        s[k] = -INFINITY;
        if (!t->live[g]) continue;
        double d[3] = {q[0] - t->mu[3 * g], q[1] - t->mu[3 * g + 1], q[2] - t->mu[3 * g + 2]};
        double Lm[3][3];
        memcpy(Lm, Lc + 9 * g, sizeof(Lm));
        s[k] = log(t->pi[g]) - 0.5 * ld[g] - 0.5 * maha2(Lm, d);
        if (s[k] > smax) smax = s[k];
      }
      double den = 0.0;
      for (int k = 0; k < 8; ++k)
        if (t->live[base + k]) den += exp(s[k] - smax);
      for (int k = 0; k < 8; ++k) {
        const int64_t g = base + k;
        if (!t->live[g]) continue;
        const double e = pe * exp(s[k] - smax) / den;
        const double m = fabs(e - tau) / tau;
        if (m < mg) mg = m;
        if (e >= tau) { st_g[top] = g; st_l[top] = cl; st_e[top] = e; ++top; }
      }
      /* next followed node: stop nodes accumulate, others are expanded */
      int expanded = 0;
      while (top > 0 && !expanded) {
        --top;
        const int64_t g = st_g[top];
        const int l = st_l[top];
        const double e = st_e[top];
        const int stop = (t->kappa[g] <= lambda_c) || (l == L - 1) || !t->has_children[g];
        if (!stop) { parent = g; plev = l; pe = e; expanded = 1; break; }
        double d[3] = {q[0] - t->mu[3 * g], q[1] - t->mu[3 * g + 1], q[2] - t->mu[3 * g + 2]};
        double Lm[3][3];
        memcpy(Lm, Lc + 9 * g, sizeof(Lm));
        const double m2 = maha2(Lm, d);
        if (bins) {
          double *b = bins + 6 * g;
          b[0] += e;
          b[1] += e * q[0];
          b[2] += e * q[1];
          b[3] += e * q[2];
          b[4] += e;
          b[5] += e * m2;
        }
        ll += e * (log(t->pig[g]) - 0.5 * ld[g] - 0.5 * m2 - 1.5 * LOG_2PI);
        ++ns;
      }
      if (!expanded) break;
    }
    if (margin) margin[i] = mg;
    if (stops) stops[i] = ns;
  }
  if (loglik) *loglik = ll / (double)n;
  free(st_g);
  free(st_l);
  free(st_e);
  free(Lc);
  free(ld);
  return OT_OK;
}

/* Registration with the soft multi-path E-step: the EM loop of oracle_register. */
int oracle_register_soft(const ot_tree *t, const float *xyz, int64_t n, double lambda_c, double tau, int max_iters,
                         double tol_rot, double tol_trans, double R[9], double tv[3], int *iters, double *loglik) {
  if (n < 1 || max_iters < 1 || !(tau > 0.0)) return OT_EINVAL;
  double *bins = (double *)malloc(sizeof(double) * 6 * (size_t)t->n_nodes);
  int st = OT_OK, it;
  double ll = 0.0;
  *iters = 0;
  for (it = 1; it <= max_iters; ++it) {
    st = oracle_estep_soft(t, xyz, n, R, tv, lambda_c, tau, bins, &ll, NULL, NULL);
    if (st != OT_OK) break;
    double H[36], g[6], x[6] = {0, 0, 0, 0, 0, 0};
    oracle_normal_equations(t, bins, n, H, g);
    *iters = it;
    st = oracle_solve_update(H, g, t->origin, R, tv, x);
    if (st != OT_OK) break;
    double wn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double tn = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
    if (wn < tol_rot && tn < tol_trans) break;
  }
  if (loglik) *loglik = ll;
  free(bins);
  return st;
}
