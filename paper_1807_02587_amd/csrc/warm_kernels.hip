// Learned warm start: coarse-GMM features, a BF16-MFMA multilayer perceptron
// (forward, backward, Adam) and the 6D-rotation head.
//
// Features of a cloud are the 64 nodes of level 1 of its GMM tree, each
// (global weight, mean (3), upper covariance (6)), expressed in the cloud's
// canonical frame: centred on the cloud mean, scaled by its RMS radius and
// rotated into its principal axes (proper rotation).  A pair's input row is
// [source 640 | target 640].  The network predicts the transform between the
// two canonical frames: a 6D rotation (first two columns, Gram-Schmidt) and a
// translation.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hgmm_dev.h"
#include "hgmm_warm.h"

namespace hgmm {

// ---------------------------------------------------------------------------
// bf16 helpers (storage as raw 16-bit, round to nearest even)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// canonical frame and features of level 1 of a tree
// ---------------------------------------------------------------------------

// frame[13]: E (3x3, rows = principal axes, det +1), centre c (3), RMS radius s
__device__ inline void canonical_frame(const TreeDev& T, double reg_eps, double* fr) {
  for (int i = 0; i < 9; ++i) fr[i] = T.root_evec[i];
  const double* e = T.root_evec;
  const double det = e[0] * (e[4] * e[8] - e[5] * e[7]) - e[1] * (e[3] * e[8] - e[5] * e[6]) +
                     e[2] * (e[3] * e[7] - e[4] * e[6]);
  if (det < 0.0) { fr[6] = -fr[6]; fr[7] = -fr[7]; fr[8] = -fr[8]; }
  for (int i = 0; i < 3; ++i) fr[9 + i] = T.origin[i];
  const double tr = T.root_cov[0] + T.root_cov[3] + T.root_cov[5] - 3.0 * reg_eps;
  fr[12] = sqrt(fmax(tr, 1e-300));
}

// One block of 64 threads per tree: lane k writes node k of level 1.
__global__ __launch_bounds__(64) void features_kernel(const int* __restrict__ tree_ids, int ntrees,
                                                     const TreeDev* __restrict__ trees, const NodeD* __restrict__ nodes,
                                                     double reg_eps, float* feat, double* frames) {
  const int b = blockIdx.x;
  if (b >= ntrees) return;
  const TreeDev& T = trees[tree_ids[b]];
  double fr[13];
  canonical_frame(T, reg_eps, fr);
  if (threadIdx.x == 0)
    for (int i = 0; i < 13; ++i) frames[(size_t)b * 13 + i] = fr[i];
  const int k = threadIdx.x;
  float* out = feat + (size_t)b * 640 + (size_t)k * 10;
  if (T.levels < 2) {
    for (int i = 0; i < 10; ++i) out[i] = 0.f;
    return;
  }
  const NodeD& n = nodes[T.node_base + 8 + k];
  if (!n.live) {
    for (int i = 0; i < 10; ++i) out[i] = 0.f;
    return;
  }
  const double is = 1.0 / fr[12];
  double d[3] = {n.mu[0] - fr[9], n.mu[1] - fr[10], n.mu[2] - fr[11]};
  double m[3];
  for (int r = 0; r < 3; ++r) m[r] = (fr[3 * r] * d[0] + fr[3 * r + 1] * d[1] + fr[3 * r + 2] * d[2]) * is;
  const double S[3][3] = {{n.cov[0], n.cov[1], n.cov[2]}, {n.cov[1], n.cov[3], n.cov[4]}, {n.cov[2], n.cov[4], n.cov[5]}};
  double ES[3][3], C[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) ES[r][c] = fr[3 * r] * S[0][c] + fr[3 * r + 1] * S[1][c] + fr[3 * r + 2] * S[2][c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      C[r][c] = (ES[r][0] * fr[3 * c] + ES[r][1] * fr[3 * c + 1] + ES[r][2] * fr[3 * c + 2]) * is * is;
  out[0] = (float)n.pig;
  out[1] = (float)m[0]; out[2] = (float)m[1]; out[3] = (float)m[2];
  out[4] = (float)C[0][0]; out[5] = (float)C[0][1]; out[6] = (float)C[0][2];
  out[7] = (float)C[1][1]; out[8] = (float)C[1][2]; out[9] = (float)C[2][2];
}

// X[p] = [feat[src_slot[p]] | feat[tgt_slot[p]]] in bf16 (1280 per row)
__global__ void assemble_kernel(const float* __restrict__ feat, const int* __restrict__ src_slot,
                                const int* __restrict__ tgt_slot, int P, uint16_t* X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)P * 1280) return;
  const int p = (int)(i / 1280), c = (int)(i % 1280);
  const int slot = c < 640 ? src_slot[p] : tgt_slot[p];
  X[i] = f2bf(feat[(size_t)slot * 640 + (c % 640)]);
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ a, uint16_t* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}

// ---------------------------------------------------------------------------
// GEMM: C[M x N] (FP32) = op(A)[M x K] * op(B)[K x N], bf16 operands, FP32
// accumulation on v_mfma_f32_16x16x32_bf16.  op(A)(i,k) = TA ? A[k*lda+i] :
// A[i*lda+k]; op(B)(k,j) = TB ? B[j*ldb+k] : B[k*ldb+j].  beta != 0 adds
// into C.  Block tile 64x64x32, 4 waves of 32x32; the tiles are staged with
// 16-byte loads along each operand's contiguous dimension.
// ---------------------------------------------------------------------------

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A, int lda,
                                                        const uint16_t* __restrict__ B, int ldb, float* C, int ldc,
                                                        float beta, int kslice, size_t cslice) {
  constexpr int BM = 64, BN = 64, BK = 32, PAD = 8;
  static_assert(BM * BK == 8 * 256 && BN * BK == 8 * 256, "one 8-element chunk of each tile per thread");
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][BK + PAD];   // row i, k
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][BK + PAD];   // column j, k (transposed)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  // slice z of the reduction: k in [kb, ke), written to C + z * cslice
  const int kb = (int)blockIdx.z * kslice;
  const int ke = K - kb < kslice ? K : kb + kslice;
  C += (size_t)blockIdx.z * cslice;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  // 16-byte loads need 16-byte aligned rows of whole 8-element chunks
  const bool vecA = (lda % 8) == 0 && ((uintptr_t)A & 15u) == 0u;
  const bool vecB = (ldb % 8) == 0 && ((uintptr_t)B & 15u) == 0u;
  f32x4_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += BK) {
    // stage the tiles: each thread moves one chunk of 8 elements of each
    // operand along its contiguous dimension, with one 16-byte load when the
    // chunk is whole and aligned, element loads at the edges
    {
      union { uint4 q; uint16_t h[8]; } u;
      if (!TA) {  // A row-major: 8 consecutive k of row i
        const int i = tid >> 2, kc = (tid & 3) * 8, gi = m0 + i, gk = k0 + kc;
        if (vecA && gi < M && gk + 8 <= ke) {
          u.q = *reinterpret_cast<const uint4*>(A + (size_t)gi * lda + gk);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) u.h[e] = (gi < M && gk + e < ke) ? A[(size_t)gi * lda + gk + e] : (uint16_t)0;
        }
        *reinterpret_cast<uint4*>(&As[i][kc]) = u.q;
      } else {  // A stored transposed: 8 consecutive i of column k
        const int k = tid >> 3, ic = (tid & 7) * 8, gk = k0 + k, gi = m0 + ic;
        if (vecA && gk < ke && gi + 8 <= M) {
          u.q = *reinterpret_cast<const uint4*>(A + (size_t)gk * lda + gi);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) u.h[e] = (gk < ke && gi + e < M) ? A[(size_t)gk * lda + gi + e] : (uint16_t)0;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) As[ic + e][k] = u.h[e];
      }
      if (TB) {  // B stored transposed: 8 consecutive k of column j
        const int j = tid >> 2, kc = (tid & 3) * 8, gj = n0 + j, gk = k0 + kc;
        if (vecB && gj < N && gk + 8 <= ke) {
          u.q = *reinterpret_cast<const uint4*>(B + (size_t)gj * ldb + gk);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) u.h[e] = (gj < N && gk + e < ke) ? B[(size_t)gj * ldb + gk + e] : (uint16_t)0;
        }
        *reinterpret_cast<uint4*>(&Bs[j][kc]) = u.q;
      } else {  // B row-major: 8 consecutive j of row k
        const int k = tid >> 3, jc = (tid & 7) * 8, gk = k0 + k, gj = n0 + jc;
        if (vecB && gk < ke && gj + 8 <= N) {
          u.q = *reinterpret_cast<const uint4*>(B + (size_t)gk * ldb + gj);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) u.h[e] = (gk < ke && gj + e < N) ? B[(size_t)gk * ldb + gj + e] : (uint16_t)0;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[jc + e][k] = u.h[e];
      }
    }
    __syncthreads();
    // A operand: row (lane % 16), k = 8*(lane/16) .. +7; B operand: column (lane % 16), same k
    const int r = lane & 15, kq = (lane >> 4) * 8;
    bf16x8_t av[2], bv[2];
    for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const bf16x8_t*>(&As[wm + 16 * a + r][kq]);
    for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const bf16x8_t*>(&Bs[wn + 16 * b + r][kq]);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  // D layout: lane holds rows 4*(lane/16) + e, column lane % 16
  const int cj = lane & 15, ri = (lane >> 4) * 4;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 4; ++e) {
        const int gi = m0 + wm + 16 * a + ri + e, gj = n0 + wn + 16 * b + cj;
        if (gi < M && gj < N) {
          float* c = C + (size_t)gi * ldc + gj;
          *c = (beta != 0.f ? beta * *c : 0.f) + acc[a][b][e];
        }
      }
}

// ---------------------------------------------------------------------------
// elementwise pieces of the MLP
// ---------------------------------------------------------------------------

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Z = C + bias (kept for the backward), H = gelu(Z) in bf16 (or Z itself for the head)
__global__ void bias_act_kernel(float* Z, const float* __restrict__ bias, int M, int N, uint16_t* H, int act) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const float z = Z[i] + bias[i % N];
  Z[i] = z;
  if (H) H[i] = f2bf(act ? gelu(z) : z);
}

// dZ = dH * gelu'(Z) -> bf16
__global__ void gelu_back_kernel(const float* __restrict__ dH, const float* __restrict__ Z, int64_t n, uint16_t* dZ,
                                 float* dZf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = dH[i] * gelu_grad(Z[i]);
  dZ[i] = f2bf(g);
  if (dZf) dZf[i] = g;
}

// db[j] = sum_i dZ[i, j] in a fixed order: a block of kColsumThreads takes
// kColsumCols columns; thread (row group g, column c) sums column c over the
// rows g, g + kColsumGroups, ... (a wave reads 4 rows of 16 consecutive
// columns at a time), and the group sums of a column are added in group order.
constexpr int kColsumThreads = 1024;
constexpr int kColsumCols = 16;
constexpr int kColsumGroups = kColsumThreads / kColsumCols;
__global__ __launch_bounds__(kColsumThreads) void colsum_kernel(const float* __restrict__ dZ, int M, int N,
                                                                float* db) {
  __shared__ float part[kColsumGroups][kColsumCols];
  const int c = threadIdx.x % kColsumCols, rg = threadIdx.x / kColsumCols;
  const int j = blockIdx.x * kColsumCols + c;
  float s = 0.f;
  if (j < N)
    for (int i = rg; i < M; i += kColsumGroups) s += dZ[(size_t)i * N + j];
  part[rg][c] = s;
  __syncthreads();
  if (rg == 0 && j < N) {
    float t = part[0][c];
    for (int g = 1; g < kColsumGroups; ++g) t += part[g][c];
    db[j] = t;
  }
}

// head loss: L = mean_p sum_c w_c (y - t)^2 / 2 (w = 1 for the 6D part, wt for
// the translation); dY = w (y - t) / P; per-row loss written to rowloss
__global__ void head_loss_kernel(const float* __restrict__ Y, const float* __restrict__ T, int P, float wt, float* dY,
                                 uint16_t* dYb, float* rowloss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float l = 0.f;
  for (int c = 0; c < 9; ++c) {
    const float w = c < 6 ? 1.f : wt;
    const float d = Y[p * 9 + c] - T[p * 9 + c];
    l += 0.5f * w * d * d;
    const float g = w * d / (float)P;
    dY[p * 9 + c] = g;
    dYb[p * 9 + c] = f2bf(g);
  }
  rowloss[p] = l;
}

// Adam on FP32 master weights; bf16 copy refreshed
__global__ void adam_kernel(float* w, float* m, float* v, const float* __restrict__ g, int64_t n, float lr, float b1,
                            float b2, float eps, float bc1, float bc2, uint16_t* wb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  w[i] = wi;
  if (wb) wb[i] = f2bf(wi);
}

// 6D + translation (canonical frames) -> FP64 pose in the clouds' frames:
// R = Es^T Rc Et, t = s_s Es^T tc + c_s - R c_t
__global__ void head_pose_kernel(const float* __restrict__ Y, const double* __restrict__ fr_src,
                                 const double* __restrict__ fr_tgt, int P, double* R0, double* t0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float* y = Y + (size_t)p * 9;
  double a[3] = {y[0], y[1], y[2]}, b[3] = {y[3], y[4], y[5]};
  double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  if (!(na > 1e-12)) { a[0] = 1; a[1] = 0; a[2] = 0; na = 1; }
  double c1[3] = {a[0] / na, a[1] / na, a[2] / na};
  double d = c1[0] * b[0] + c1[1] * b[1] + c1[2] * b[2];
  double c2[3] = {b[0] - d * c1[0], b[1] - d * c1[1], b[2] - d * c1[2]};
  double nb = sqrt(c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2]);
  if (!(nb > 1e-12)) {
    // any unit vector orthogonal to c1
    double h[3] = {fabs(c1[0]) < 0.9 ? 1.0 : 0.0, fabs(c1[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    double dd = c1[0] * h[0] + c1[1] * h[1] + c1[2] * h[2];
    c2[0] = h[0] - dd * c1[0]; c2[1] = h[1] - dd * c1[1]; c2[2] = h[2] - dd * c1[2];
    nb = sqrt(c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2]);
  }
  for (int i = 0; i < 3; ++i) c2[i] /= nb;
  double c3[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2], c1[0] * c2[1] - c1[1] * c2[0]};
  // Rc columns c1, c2, c3
  double Rc[3][3];
  for (int i = 0; i < 3; ++i) { Rc[i][0] = c1[i]; Rc[i][1] = c2[i]; Rc[i][2] = c3[i]; }
  const double* Es = fr_src + (size_t)p * 13;
  const double* Et = fr_tgt + (size_t)p * 13;
  double M1[3][3], R[3][3];
  for (int i = 0; i < 3; ++i)  // M1 = Rc Et
    for (int j = 0; j < 3; ++j) M1[i][j] = Rc[i][0] * Et[j] + Rc[i][1] * Et[3 + j] + Rc[i][2] * Et[6 + j];
  for (int i = 0; i < 3; ++i)  // R = Es^T M1
    for (int j = 0; j < 3; ++j) R[i][j] = Es[i] * M1[0][j] + Es[3 + i] * M1[1][j] + Es[6 + i] * M1[2][j];
  const double tc[3] = {y[6], y[7], y[8]};
  const double ss = Es[12];
  for (int i = 0; i < 3; ++i) {
    double v = ss * (Es[i] * tc[0] + Es[3 + i] * tc[1] + Es[6 + i] * tc[2]) + Es[9 + i];
    v -= R[i][0] * Et[9] + R[i][1] * Et[10] + R[i][2] * Et[11];
    t0[3 * p + i] = v;
    for (int j = 0; j < 3; ++j) R0[9 * p + 3 * i + j] = R[i][j];
  }
}

// canonical training target from a pose: Rc = Es R Et^T, tc = Es (R c_t + t - c_s) / s_s;
// row = [Rc col 0 (3), Rc col 1 (3), tc (3)]
__global__ void head_target_kernel(const double* __restrict__ R, const double* __restrict__ t,
                                   const double* __restrict__ fr_src, const double* __restrict__ fr_tgt, int P,
                                   float* T) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double* Es = fr_src + (size_t)p * 13;
  const double* Et = fr_tgt + (size_t)p * 13;
  const double* Rp = R + 9 * (size_t)p;
  double M1[3][3], Rc[3][3];
  for (int i = 0; i < 3; ++i)  // M1 = R Et^T
    for (int j = 0; j < 3; ++j) M1[i][j] = Rp[3 * i] * Et[3 * j] + Rp[3 * i + 1] * Et[3 * j + 1] + Rp[3 * i + 2] * Et[3 * j + 2];
  for (int i = 0; i < 3; ++i)  // Rc = Es M1
    for (int j = 0; j < 3; ++j) Rc[i][j] = Es[3 * i] * M1[0][j] + Es[3 * i + 1] * M1[1][j] + Es[3 * i + 2] * M1[2][j];
  double w[3];
  for (int i = 0; i < 3; ++i)
    w[i] = Rp[3 * i] * Et[9] + Rp[3 * i + 1] * Et[10] + Rp[3 * i + 2] * Et[11] + t[3 * p + i] - Es[9 + i];
  float* o = T + (size_t)p * 9;
  for (int i = 0; i < 3; ++i) { o[i] = (float)Rc[i][0]; o[3 + i] = (float)Rc[i][1]; }
  for (int i = 0; i < 3; ++i) o[6 + i] = (float)((Es[3 * i] * w[0] + Es[3 * i + 1] * w[1] + Es[3 * i + 2] * w[2]) / Es[12]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_features(const int* tree_ids, int ntrees, const TreeDev* trees, const NodeD* nodes, double reg_eps,
                     float* feat, double* frames, hipStream_t s) {
  if (ntrees <= 0) return;
  hipLaunchKernelGGL(features_kernel, dim3(ntrees), dim3(64), 0, s, tree_ids, ntrees, trees, nodes, reg_eps, feat,
                     frames);
}

void launch_assemble(const float* feat, const int* src_slot, const int* tgt_slot, int P, uint16_t* X, hipStream_t s) {
  hipLaunchKernelGGL(assemble_kernel, dim3(nblk((int64_t)P * 1280, 256)), dim3(256), 0, s, feat, src_slot, tgt_slot, P,
                     X);
}

void launch_f32_to_bf16(const float* a, uint16_t* b, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, a, b, n);
}

void launch_gemm(bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                 float* C, int ldc, float beta, hipStream_t s) {
  launch_gemm_slices(ta, tb, M, N, K, A, lda, B, ldb, C, ldc, beta, 1, s);
}

void launch_gemm_slices(bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                        float* C, int ldc, float beta, int slices, hipStream_t s) {
  // slices of the reduction in whole 32-element K steps (16-byte loads stay
  // aligned); slice z writes C + z * M * ldc
  const int steps = (K + 31) / 32;
  const int per = slices > 1 ? (steps + slices - 1) / slices : steps;
  const int nz = slices > 1 ? (steps + per - 1) / per : 1;
  const int kslice = slices > 1 ? 32 * per : K;
  const size_t cslice = (size_t)M * (size_t)ldc;
  dim3 grid((N + 63) / 64, (M + 63) / 64, (unsigned)(nz > 0 ? nz : 1));
  if (!ta && !tb) hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, beta, kslice, cslice);
  else if (!ta && tb) hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, beta, kslice, cslice);
  else if (ta && !tb) hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, beta, kslice, cslice);
  else hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, beta, kslice, cslice);
}

// out[e] = sum over the slices of part[z * n + e], in slice order
__global__ void sum_slices_kernel(const float* __restrict__ part, int slices, int64_t n, float* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float t = part[e];
  for (int z = 1; z < slices; ++z) t += part[(size_t)z * (size_t)n + (size_t)e];
  out[e] = t;
}

void launch_sum_slices(const float* part, int slices, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(sum_slices_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, part, slices, n, out);
}

void launch_bias_act(float* Z, const float* bias, int M, int N, uint16_t* H, int act, hipStream_t s) {
  hipLaunchKernelGGL(bias_act_kernel, dim3(nblk((int64_t)M * N, 256)), dim3(256), 0, s, Z, bias, M, N, H, act);
}

void launch_gelu_back(const float* dH, const float* Z, int64_t n, uint16_t* dZ, float* dZf, hipStream_t s) {
  hipLaunchKernelGGL(gelu_back_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, dH, Z, n, dZ, dZf);
}

void launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((N + kColsumCols - 1) / kColsumCols)), dim3(kColsumThreads), 0, s,
                     dZ, M, N, db);
}

void launch_head_loss(const float* Y, const float* T, int P, float wt, float* dY, uint16_t* dYb, float* rowloss,
                      hipStream_t s) {
  hipLaunchKernelGGL(head_loss_kernel, dim3(nblk(P, 256)), dim3(256), 0, s, Y, T, P, wt, dY, dYb, rowloss);
}

void launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, uint16_t* wb, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, eps, bc1, bc2, wb);
}

void launch_head_pose(const float* Y, const double* fr_src, const double* fr_tgt, int P, double* R0, double* t0,
                      hipStream_t s) {
  hipLaunchKernelGGL(head_pose_kernel, dim3(nblk(P, 128)), dim3(128), 0, s, Y, fr_src, fr_tgt, P, R0, t0);
}

void launch_head_target(const double* R, const double* t, const double* fr_src, const double* fr_tgt, int P, float* T,
                        hipStream_t s) {
  hipLaunchKernelGGL(head_target_kernel, dim3(nblk(P, 128)), dim3(128), 0, s, R, t, fr_src, fr_tgt, P, T);
}

}  // namespace hgmm
