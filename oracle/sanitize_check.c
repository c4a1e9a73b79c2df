/*
 * Host sanitizer run of the FP64 oracle (test infrastructure only, like the
 * oracle itself).  Built with -fsanitize=address,undefined by
 * tests/test_oracle_sanitizers.py, it builds a 3-level tree of a small
 * synthetic cloud (three planes and a sphere in the unit cube), then runs the
 * E-step and the registration of each association the oracle implements:
 * the adaptive descent, the single-level mixture of level 1 and the soft
 * multi-path descent, each with every optional output requested so that every
 * write path is exercised.  Any out-of-bounds access, leak or undefined
 * behaviour aborts the run; otherwise it exits 0 when every call returned
 * OT_OK and every output is finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "hgmm_oracle.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;

/* uniform in [0, 1): 53 bits of a 64-bit linear congruential generator */
static double urand(void) {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static int fail(const char *what, int rc) {
  fprintf(stderr, "sanitize_check: %s returned %d\n", what, rc);
  return 1;
}

static int finite_all(const double *v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

int main(void) {
  const int64_t n = 3000;
  const int levels = 3;
  float *xyz = (float *)malloc(sizeof(float) * 3 * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {urand(), urand(), urand()};
    const double noise = 0.002 * (urand() - 0.5);
    switch (i % 4) {
      case 0: p[2] = 0.2 + noise; break;
      case 1: p[0] = 0.8 + noise; break;
      case 2: p[1] = 0.5 + noise; break;
      default: {
        /* a point on the sphere of radius 0.2 around the cube's centre */
        double d[3] = {p[0] - 0.5, p[1] - 0.5, p[2] - 0.5};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r < 1e-9) r = 1e-9;
        for (int k = 0; k < 3; ++k) p[k] = 0.5 + (0.2 + noise) * d[k] / r;
      }
    }
    for (int k = 0; k < 3; ++k) xyz[(size_t)k * (size_t)n + (size_t)i] = (float)p[k];
  }

  ot_tree t = {0};
  const int64_t nn = oracle_level_offset(levels);
  t.levels = levels;
  t.n_nodes = nn;
  t.live = (int32_t *)calloc((size_t)nn, sizeof(int32_t));
  t.has_children = (int32_t *)calloc((size_t)nn, sizeof(int32_t));
  t.count = (int64_t *)calloc((size_t)nn, sizeof(int64_t));
  t.pi = (double *)calloc((size_t)nn, sizeof(double));
  t.pig = (double *)calloc((size_t)nn, sizeof(double));
  t.mu = (double *)calloc(3 * (size_t)nn, sizeof(double));
  t.cov = (double *)calloc(6 * (size_t)nn, sizeof(double));
  t.lam = (double *)calloc(3 * (size_t)nn, sizeof(double));
  t.evec = (double *)calloc(9 * (size_t)nn, sizeof(double));
  t.kappa = (double *)calloc((size_t)nn, sizeof(double));
  int32_t *labels = (int32_t *)malloc(sizeof(int32_t) * (size_t)levels * (size_t)n);
  int bad = 0;
  int rc = oracle_build(xyz, n, levels, 10, 1e-6, 1.0, &t, labels);
  if (rc != OT_OK) return fail("oracle_build", rc);
  int64_t live = 0;
  for (int64_t g = 0; g < nn; ++g) live += t.live[g] != 0;
  if (live < 8 + 64) return fail("oracle_build (too few live nodes)", (int)live);

  /* a 2 degree rotation about (0.3, -1, 0.4) and a small shift */
  const double ax[3] = {0.3 / 1.1180339887498949, -1.0 / 1.1180339887498949, 0.4 / 1.1180339887498949};
  const double th = 2.0 * 3.14159265358979323846 / 180.0, c = cos(th), s = sin(th);
  double R0[9], t0[3] = {0.003, -0.002, 0.001};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double K = (i == j) ? 0.0 : (i == 0 && j == 1) ? -ax[2] : (i == 0 && j == 2) ? ax[1]
                       : (i == 1 && j == 0) ? ax[2] : (i == 1 && j == 2) ? -ax[0] : (i == 2 && j == 0) ? -ax[1] : ax[0];
      R0[3 * i + j] = (i == j ? c : 0.0) + s * K + (1.0 - c) * ax[i] * ax[j];
    }

  int32_t *stop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *stop_level = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double *gamma = (double *)malloc(sizeof(double) * (size_t)n);
  double *gap = (double *)malloc(sizeof(double) * (size_t)n);
  double *bins = (double *)malloc(sizeof(double) * 6 * (size_t)nn);
  double *margin = (double *)malloc(sizeof(double) * (size_t)n);
  double *trace = (double *)malloc(sizeof(double) * 20 * 8);
  double ll = 0.0;
  double R[9], tv[3];
  int iters = 0;

  rc = oracle_estep(&t, xyz, n, R0, t0, 0.01, stop, stop_level, gamma, gap, bins, &ll);
  if (rc != OT_OK) bad |= fail("oracle_estep", rc);
  bad |= !finite_all(gamma, n) || !isfinite(ll);
  for (int k = 0; k < 9; ++k) R[k] = R0[k];
  for (int k = 0; k < 3; ++k) tv[k] = t0[k];
  rc = oracle_register(&t, xyz, n, 8, 0.01, 1e-9, 1e-9, R, tv, &iters, &ll, trace);
  if (rc != OT_OK) bad |= fail("oracle_register", rc);
  bad |= !finite_all(R, 9) || !finite_all(tv, 3);

  rc = oracle_estep_flat(&t, 1, xyz, n, R0, t0, stop, gamma, gap, bins, &ll);
  if (rc != OT_OK) bad |= fail("oracle_estep_flat", rc);
  bad |= !finite_all(gamma, n) || !isfinite(ll);
  for (int k = 0; k < 9; ++k) R[k] = R0[k];
  for (int k = 0; k < 3; ++k) tv[k] = t0[k];
  rc = oracle_register_flat(&t, 1, xyz, n, 6, 1e-9, 1e-9, R, tv, &iters, &ll);
  if (rc != OT_OK) bad |= fail("oracle_register_flat", rc);
  bad |= !finite_all(R, 9) || !finite_all(tv, 3);

  rc = oracle_estep_soft(&t, xyz, n, R0, t0, 0.01, 0.05, bins, &ll, margin, stop);
  if (rc != OT_OK) bad |= fail("oracle_estep_soft", rc);
  bad |= !finite_all(bins, 6 * nn) || !isfinite(ll);
  for (int k = 0; k < 9; ++k) R[k] = R0[k];
  for (int k = 0; k < 3; ++k) tv[k] = t0[k];
  rc = oracle_register_soft(&t, xyz, n, 0.01, 0.05, 4, 1e-9, 1e-9, R, tv, &iters, &ll);
  if (rc != OT_OK) bad |= fail("oracle_register_soft", rc);
  bad |= !finite_all(R, 9) || !finite_all(tv, 3);

  free(xyz); free(labels); free(stop); free(stop_level); free(gamma); free(gap); free(bins); free(margin);
  free(trace);
  free(t.live); free(t.has_children); free(t.count); free(t.pi); free(t.pig); free(t.mu); free(t.cov);
  free(t.lam); free(t.evec); free(t.kappa);
  if (bad) {
    fprintf(stderr, "sanitize_check: a call failed or gave a non-finite output\n");
    return 1;
  }
  printf("sanitize_check: ok (%lld live nodes of %lld, last registration %d iterations)\n", (long long)live,
         (long long)nn, iters);
  return 0;
}
