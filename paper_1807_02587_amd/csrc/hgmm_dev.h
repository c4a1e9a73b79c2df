// Device-side data layout and helpers shared by the build and registration
// kernels of the GMM-Tree library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hgmm {

constexpr int kMaxLevels = 6;
constexpr int kBlock = 256;                              // threads per block of the point kernels
constexpr double kLog2e = 1.4426950408889634;            // scores are kept in log2 units
constexpr double kWScale = 0.84932180028801904272;       // sqrt(0.5 * log2(e))
constexpr float kU = 5.9604644775390625e-8f;             // unit roundoff of FP32, 2^-24
constexpr double kLog2Pi = 1.8378770664093453;

enum : uint32_t { F_LIVE = 1u, F_STOP = 2u, F_HASCH = 4u };

// FP64 record of one tree node.  mu is in absolute model coordinates; cov
// includes the eps*I regularisation; winv is the inverse of the lower Cholesky
// factor of cov, packed [00, 10, 11, 20, 21, 22]; c = log(pi) - log|cov|/2
// with pi the weight inside the sibling group.  The FP64 scoring fields (mu,
// winv, c) come first, 80 contiguous bytes (NodeS).
struct NodeD {
  double mu[3];
  double winv[6];
  double c;
  double cov[6];
  double lam[3];
  double evec[9];
  double pi, pig, kappa, logdet;
  int32_t live, has_children;
  int64_t count;
};

// The FP64 scoring prefix of a NodeD (same layout as its first 80 bytes).
struct NodeS {
  double mu[3];
  double winv[6];
  double c;
};
static_assert(sizeof(NodeS) == 80, "NodeS is the 80-byte prefix of NodeD");
static_assert(__builtin_offsetof(NodeD, winv) == 24 && __builtin_offsetof(NodeD, c) == 72,
              "the FP64 scoring fields lead NodeD");

// FP32 scoring record of one node, 64 bytes.  The score of a point p is
//   s = c - |W d|^2,  d = float(p - mu)  (the subtraction in FP64),
// which equals log2(e) * (log pi - log|cov|/2 - Mahalanobis^2/2).
// errc and errg give a rigorous bound on the FP32 rounding of s:
//   |s_fp32 - s| <= errc + 4u q + errg * max|d| * (1 + q).
struct __align__(16) NodeF {
  double mu[3];
  float w[6];
  float c;
  uint32_t flags;
  float errc;
  float errg;
};
static_assert(sizeof(NodeF) == 64, "NodeF must be one 64-byte line");

// FP64 scoring record of one node for the tree descent, 96 bytes:
//   s = c - |W (p - mu)|^2,  W = sqrt(log2(e) / 2) * winv,  c = log2(e) * c_node,
// the score of NodeF in FP64.  A dead node has mu = 0, W = 0 and c = -inf, so
// it scores -inf for every point.
struct __align__(16) NodeR {
  double mu[3];
  double w[6];
  double c;
  uint32_t flags;
  uint32_t pad[3];
};
static_assert(sizeof(NodeR) == 96, "NodeR is six 16-byte words");

// A contiguous range of sorted points that belongs to one parent (a "job").
struct Tile {
  int32_t start, end, job, pad;
};

// One parent whose 8 children are fitted by EM at the current level.
struct Job {
  int32_t start, count;   // range of the parent's points in the sorted arrays
  int32_t parent;         // global node id of the parent, -1 for a tree root
  int32_t child_base;     // global node id of child 0
  int32_t child_lvl;      // index of child 0 in the level-compact info arrays
  int32_t tile_first, ntiles;
  int32_t tree;
};

// Per-tree constants.  The root record is written by the root kernels.
struct TreeDev {
  double origin[3];
  double extent;
  double root_cov[6];
  double root_lam[3];
  double root_evec[9];
  int64_t node_base;      // first global node id of this tree
  int64_t point_off;      // first point of this tree in the (CSR) point arrays
  int64_t label_base;     // first label of this tree: labels[label_base + l * n_points + i]
  int32_t levels;
  int32_t n_points;
  int32_t status;         // 0 or a negative hgmm_status found on the device
  int32_t pad;
};

// One tree that has a given level (levels > level): its index in the forest,
// the level-compact base of its nodes one level up (the parents; -1 at level
// 0) and at the level itself.
struct LevelTree {
  int32_t b, prev_base, cur_base, pad;
};

// Fields of a level plan made on the device (ints): jobs, tiles, tiles of the
// tiled jobs, jobs per class (block of 64 / 256 / 512 threads, tiled), start of
// each class in the class-ordered job list, points per tile, and an overflow
// flag.
enum PlanField { PL_NJOBS = 0, PL_NTILES = 1, PL_NBIG = 2, PL_CLS_N = 3, PL_CLS_OFF = 7, PL_TPTS = 12, PL_ERR = 13,
                 PL_SIZE = 16 };

// Registration state of one pair, FP64, device resident.
struct PoseState {
  double R[9];
  double t[3];
  double loglik;
  double x[6];            // last increment (omega, tau)
  int32_t iters;
  int32_t done;
  int32_t status;
  int32_t pad;
};

// Registration moments of one node in fixed point: M0 = sum gamma, D = sum
// gamma (T(p) - mu) (3 values), Q = sum of squared Mahalanobis distances, and
// the number of points.  A contribution v of value j is scaled by an exact or
// fixed factor (kFixScaleM0 for M0, kFixScaleD / extent for D, kFixScaleQ for
// Q),
// split into its integer part hi = floor(v') and 32 fractional bits
// lo = floor((v' - hi) 2^32), and the two parts are summed in separate 64-bit
// integers with no carry between them: value' = sum hi + (sum lo) 2^-32.
// Integer sums do not depend on the order of the additions, so the totals
// are the same whatever order waves, blocks and XCDs add in, and every add is
// an atomic add whose result is not needed (no round trip).  Scaled values
// are saturated at +-2^62.  96 bytes.
constexpr int kFixVals = 5;
constexpr double kFixScaleM0 = 1048576.0;  // 2^20: resolution 2^-52, range 2^42 of gamma sums
constexpr double kFixScaleD = 65536.0;     // 2^16 per extent: resolution 2^-48 extent, range 2^46 extent
constexpr double kFixScaleQ = 256.0;       // 2^8: resolution 2^-40, range 2^54 of squared distances
struct FixBin {
  unsigned long long lo[kFixVals];  // sums of 32-bit fractions
  long long hi[kFixVals];           // sums of integer parts
  unsigned long long cnt;
  unsigned long long pad;
};
static_assert(sizeof(FixBin) == 96, "FixBin is 12 words");

// ---------------------------------------------------------------------------
// wave64 reductions through DPP (all 64 lanes must be active)
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, BANK_MASK, true));
}

// Sum over the 64 lanes, returned as a wave-uniform value.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_f<0x114>(v);       // row_shr:4
  v += dpp_f<0x118>(v);       // row_shr:8   -> lane 15 of each row holds the row sum
  v += dpp_f<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3 -> lane 63 holds the total
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, BANK_MASK, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, BANK_MASK, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// FP64 sum over the 64 lanes in a fixed order, wave-uniform result.
__device__ __forceinline__ double wave_sum_dd(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x114>(v);
  v += dpp_d<0x118>(v);
  v += dpp_d<0x142, 0xA>(v);
  v += dpp_d<0x143, 0xC>(v);
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Fixed-order FP64 sum of `count` consecutive doubles starting at p, by one
// full wave (lane i takes elements i, i+64, ...).  Wave-uniform result.
__device__ __forceinline__ double wave_sum_range(const double* p, int count, int lane) {
  double s = 0.0;
  for (int i = lane; i < count; i += 64) s += p[i];
  return wave_sum_dd(s);
}

// Fixed-order FP64 totals of NV rows of `count` values each, row v starting at
// p + v * stride.  Lane l adds elements l, l + 64, l + 128, ... in that order;
// every round first issues the loads of U elements of all NV rows (NV * U
// independent loads in flight), then adds them.  Wave-uniform results.
template <int NV, int U>
__device__ __forceinline__ void wave_fold(const double* __restrict__ p, size_t stride, int count, int lane,
                                          double (&out)[NV]) {
  double s[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = 0.0;
  for (int base = 0; base < count; base += 64 * U) {
    double x[NV][U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int i = base + lane + 64 * k;
#pragma unroll
      for (int v = 0; v < NV; ++v) x[v][k] = (i < count) ? p[(size_t)v * stride + i] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int k = 0; k < U; ++k) s[v] += x[v][k];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = wave_sum_dd(s[v]);
}

// wave_fold of the partials of one node that carry a set bit in a per-partial
// mask word (bit `bit` of mask[i]).  A partial without it is an exact zero
// that was not written: it is not read and 0.0 is added in its place, so the
// sum, its order and its rounding are those of the dense fold.
template <int NV, int U>
__device__ __forceinline__ void wave_fold_masked(const double* __restrict__ p, size_t stride,
                                                 const uint64_t* __restrict__ mask, int bit, int count, int lane,
                                                 double (&out)[NV]) {
  double s[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = 0.0;
  for (int base = 0; base < count; base += 64 * U) {
    double x[NV][U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int i = base + lane + 64 * k;
      const bool on = i < count && ((mask[i] >> bit) & 1ull);
#pragma unroll
      for (int v = 0; v < NV; ++v) x[v][k] = on ? p[(size_t)v * stride + i] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int k = 0; k < U; ++k) s[v] += x[v][k];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = wave_sum_dd(s[v]);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ---------------------------------------------------------------------------
// fixed-point moments (FixBin)
// ---------------------------------------------------------------------------

// Integer part and 32 fractional bits of a scaled contribution (integer
// parts within 32 bits, the usual case, take the single-instruction
// conversion).
__device__ __forceinline__ void fix_split(double v, unsigned long long& lo, long long& hi) {
  v = fmin(fmax(v, -4611686018427387904.0), 4611686018427387904.0);
  const double f = floor(v);
  lo = (unsigned long long)(unsigned)((v - f) * 4294967296.0);  // v - f in [0, 1), exact
  hi = (fabs(f) < 2147483648.0) ? (long long)(int)f : (long long)f;
}

__device__ __forceinline__ double from_fix(unsigned long long lo, long long hi) {
  return (double)hi + (double)lo * 2.3283064365386963e-10;  // 2^-32
}

// Adds one split contribution; both words are plain 64-bit integer atomic
// adds whose results are unused.  Works on LDS and global memory.
__device__ __forceinline__ void fix_add(unsigned long long* plo, long long* phi, unsigned long long lo, long long hi) {
  if (lo != 0ull) atomicAdd(plo, lo);
  if (hi != 0ll) atomicAdd(reinterpret_cast<unsigned long long*>(phi), (unsigned long long)hi);
}

// The moments {M0, D (3), count, Q} of a fixed-point bin of a tree of the
// given extent.
__device__ __forceinline__ void fix_read(const FixBin& F, double extent, double (&b)[6]) {
  const double uD = (extent > 0.0 ? extent : 1.0) / kFixScaleD;
  b[0] = from_fix(F.lo[0], F.hi[0]) * (1.0 / kFixScaleM0);
  b[1] = from_fix(F.lo[1], F.hi[1]) * uD;
  b[2] = from_fix(F.lo[2], F.hi[2]) * uD;
  b[3] = from_fix(F.lo[3], F.hi[3]) * uD;
  b[4] = (double)F.cnt;
  b[5] = from_fix(F.lo[4], F.hi[4]) * (1.0 / kFixScaleQ);
}

// ---------------------------------------------------------------------------
// FP64 3x3 helpers
// ---------------------------------------------------------------------------

// Lower Cholesky factor L of a packed SPD matrix and its inverse (packed).
// Returns false when a pivot is not positive.  Short dependency chain for the
// per-iteration M-step: three square roots, three reciprocals and one log of
// the pivot product (log|cov| = log(p0 p1 p2) with pivots p_i = L_ii^2).
__device__ __forceinline__ bool chol_inv3(const double c[6], double winv[6], double& logdet) {
  const double p0 = c[0];
  if (!(p0 > 0.0)) return false;
  const double l00 = sqrt(p0), i00 = 1.0 / l00;
  const double l10 = c[1] * i00, l20 = c[2] * i00;
  const double p1 = c[3] - l10 * l10;
  if (!(p1 > 0.0)) return false;
  const double l11 = sqrt(p1), i11 = 1.0 / l11;
  const double l21 = (c[4] - l20 * l10) * i11;
  const double p2 = c[5] - l20 * l20 - l21 * l21;
  if (!(p2 > 0.0)) return false;
  const double l22 = sqrt(p2), i22 = 1.0 / l22;
  const double i10 = -l10 * i00 * i11;
  const double i21 = -l21 * i11 * i22;
  const double i20 = -(l20 * i00 + l21 * i10) * i22;
  winv[0] = i00; winv[1] = i10; winv[2] = i11; winv[3] = i20; winv[4] = i21; winv[5] = i22;
  logdet = log(p0 * p1 * p2);
  return true;
}

// Symmetric eigen-decomposition of a packed 3x3 matrix by cyclic Jacobi
// sweeps.  lam sorted descending; ev row r is the eigenvector of lam[r] with
// its largest-magnitude component positive (first one on equal magnitudes).
__device__ inline void eig_sym3(const double c[6], double lam[3], double ev[9]) {
  double A[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    double dia = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
    if (off <= 1e-300 || off <= 1e-20 * dia) break;
    for (int r = 0; r < 3; ++r) {
      int p = P[r], q = Q[r];
      double apq = A[p][q];
      if (apq == 0.0) continue;
      // symmetric 2x2 Schur decomposition: cot(2 phi) = (a_qq - a_pp) / (2 a_pq)
      double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
      double tn = copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
      double cs = rsqrt(1.0 + tn * tn);
      double sn = tn * cs;
      for (int k = 0; k < 3; ++k) {  // columns p, q
        double x = A[k][p], y = A[k][q];
        A[k][p] = cs * x - sn * y;
        A[k][q] = sn * x + cs * y;
        double vx = V[k][p], vy = V[k][q];
        V[k][p] = cs * vx - sn * vy;
        V[k][q] = sn * vx + cs * vy;
      }
      for (int k = 0; k < 3; ++k) {  // rows p, q
        double x = A[p][k], y = A[q][k];
        A[p][k] = cs * x - sn * y;
        A[q][k] = sn * x + cs * y;
      }
    }
  }
  double d[3] = {A[0][0], A[1][1], A[2][2]};
  int o[3] = {0, 1, 2};
  if (d[o[1]] > d[o[0]]) { int s = o[0]; o[0] = o[1]; o[1] = s; }
  if (d[o[2]] > d[o[0]]) { int s = o[0]; o[0] = o[2]; o[2] = s; }
  if (d[o[2]] > d[o[1]]) { int s = o[1]; o[1] = o[2]; o[2] = s; }
  for (int r = 0; r < 3; ++r) {
    int col = o[r];
    lam[r] = d[col];
    double e0 = V[0][col], e1 = V[1][col], e2 = V[2][col];
    double b = e0;
    if (fabs(e1) > fabs(b)) b = e1;
    if (fabs(e2) > fabs(b) && fabs(e2) > fabs(e1)) b = e2;
    double s = b < 0.0 ? -1.0 : 1.0;
    ev[3 * r] = s * e0; ev[3 * r + 1] = s * e1; ev[3 * r + 2] = s * e2;
  }
}

// Scoring parameters of a node from its FP64 mean, covariance and weight.
// Returns false when cov is not positive definite.
__device__ inline bool make_node(const double mu[3], const double cov[6], double pi, NodeD& nd, NodeF& nf) {
  double winv[6], logdet;
  if (!(pi > 0.0) || !chol_inv3(cov, winv, logdet)) return false;
  for (int i = 0; i < 3; ++i) nd.mu[i] = mu[i];
  for (int i = 0; i < 6; ++i) { nd.cov[i] = cov[i]; nd.winv[i] = winv[i]; }
  nd.pi = pi;
  nd.logdet = logdet;
  nd.c = log(pi) - 0.5 * logdet;
  nd.live = 1;
  float g = 0.f;
  for (int i = 0; i < 3; ++i) nf.mu[i] = mu[i];
  for (int i = 0; i < 6; ++i) nf.w[i] = (float)(winv[i] * kWScale);
  float r0 = fabsf(nf.w[0]);
  float r1 = fabsf(nf.w[1]) + fabsf(nf.w[2]);
  float r2 = fabsf(nf.w[3]) + fabsf(nf.w[4]) + fabsf(nf.w[5]);
  g = fmaxf(r0, fmaxf(r1, r2));
  nf.c = (float)(nd.c * kLog2e);
  nf.flags = F_LIVE;
  nf.errc = 2.f * kU * fabsf(nf.c) * 1.0001f;
  nf.errg = 9.f * kU * g * 1.0001f;
  return true;
}

// FP64 1/sqrt(x) for a positive normal x: the hardware estimate refined by
// two Newton steps (each at least doubles the number of correct bits).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// The FP32 scoring record alone (what an intermediate EM iteration needs):
// the same Cholesky inverse as chol_inv3 with the three pivots' inverse
// square roots taken directly, and one logarithm for the constant,
// log2(pi) - log2|cov| / 2 = log2(pi / (L00 L11 L22)).
__device__ inline bool make_nodef_fast(const double mu[3], const double c[6], double pi, NodeF& nf) {
  const double p0 = c[0];
  if (!(pi > 0.0) || !(p0 > 0.0)) return false;
  const double i00 = rsqrt_nr(p0);
  const double l10 = c[1] * i00, l20 = c[2] * i00;
  const double p1 = c[3] - l10 * l10;
  if (!(p1 > 0.0)) return false;
  const double i11 = rsqrt_nr(p1);
  const double l21 = (c[4] - l20 * l10) * i11;
  const double p2 = c[5] - l20 * l20 - l21 * l21;
  if (!(p2 > 0.0)) return false;
  const double i22 = rsqrt_nr(p2);
  const double i10 = -l10 * i00 * i11;
  const double i21 = -l21 * i11 * i22;
  const double i20 = -(l20 * i00 + l21 * i10) * i22;
  const double winv[6] = {i00, i10, i11, i20, i21, i22};
  for (int i = 0; i < 3; ++i) nf.mu[i] = mu[i];
  for (int i = 0; i < 6; ++i) nf.w[i] = (float)(winv[i] * kWScale);
  const float r0 = fabsf(nf.w[0]);
  const float r1 = fabsf(nf.w[1]) + fabsf(nf.w[2]);
  const float r2 = fabsf(nf.w[3]) + fabsf(nf.w[4]) + fabsf(nf.w[5]);
  const float g = fmaxf(r0, fmaxf(r1, r2));
  nf.c = (float)log2(pi * i00 * i11 * i22);
  nf.flags = F_LIVE;
  nf.errc = 2.f * kU * fabsf(nf.c) * 1.0001f;
  nf.errg = 9.f * kU * g * 1.0001f;
  return true;
}

// FP32 score of a node for a point given in FP64, with the pieces of the
// rounding bound.
__device__ __forceinline__ float score32(const NodeF& t, double p0, double p1, double p2, float& q, float& m) {
  float d0 = (float)(p0 - t.mu[0]);
  float d1 = (float)(p1 - t.mu[1]);
  float d2 = (float)(p2 - t.mu[2]);
  float w0 = t.w[0] * d0;
  float w1 = fmaf(t.w[1], d0, t.w[2] * d1);
  float w2 = fmaf(t.w[3], d0, fmaf(t.w[4], d1, t.w[5] * d2));
  q = fmaf(w0, w0, fmaf(w1, w1, w2 * w2));
  m = fmaxf(fabsf(d0), fmaxf(fabsf(d1), fabsf(d2)));
  return t.c - q;
}

__device__ __forceinline__ float score_err(const NodeF& t, float q, float m) {
  float gm = t.errg * m;
  return t.errc + 4.f * kU * q + fmaf(gm, q, gm);
}

// FP64 score in the same log2 units, from the FP64 scoring fields.
template <typename N>
__device__ __forceinline__ double score64(const N& n, double p0, double p1, double p2) {
  double d0 = p0 - n.mu[0], d1 = p1 - n.mu[1], d2 = p2 - n.mu[2];
  double w0 = n.winv[0] * d0;
  double w1 = n.winv[1] * d0 + n.winv[2] * d1;
  double w2 = n.winv[3] * d0 + n.winv[4] * d1 + n.winv[5] * d2;
  return kLog2e * (n.c - 0.5 * (w0 * w0 + w1 * w1 + w2 * w2));
}

// The squared whitened offset |W (p - mu)|^2 of a NodeR (in any address
// space), which is
// log2(e) / 2 times the squared Mahalanobis distance.
template <typename N>
__device__ __forceinline__ double quad_r(const N& n, double p0, double p1, double p2) {
  const double d0 = p0 - n.mu[0], d1 = p1 - n.mu[1], d2 = p2 - n.mu[2];
  const double w0 = n.w[0] * d0;
  const double w1 = fma(n.w[1], d0, n.w[2] * d1);
  const double w2 = fma(n.w[3], d0, fma(n.w[4], d1, n.w[5] * d2));
  return fma(w0, w0, fma(w1, w1, w2 * w2));
}

}  // namespace hgmm
