// Launchers of the warm-start kernels (features, bf16 MFMA GEMM, MLP pieces).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hgmm_dev.h"

namespace hgmm {

void launch_features(const int* tree_ids, int ntrees, const TreeDev* trees, const NodeD* nodes, double reg_eps,
                     float* feat, double* frames, hipStream_t s);
void launch_assemble(const float* feat, const int* src_slot, const int* tgt_slot, int P, uint16_t* X, hipStream_t s);
void launch_f32_to_bf16(const float* a, uint16_t* b, int64_t n, hipStream_t s);
void launch_gemm(bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                 float* C, int ldc, float beta, hipStream_t s);
// The same product with the reduction split into `slices` parts (whole
// 32-element steps; fewer when K is short): slice z writes its partial
// product to C + z * M * ldc.  The number of slices used is
// gemm_slices_used(K, slices).
void launch_gemm_slices(bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                        float* C, int ldc, float beta, int slices, hipStream_t s);
// out[e] = sum of part[z * n + e] over z = 0 .. slices - 1, in that order.
void launch_sum_slices(const float* part, int slices, int64_t n, float* out, hipStream_t s);
inline int gemm_slices_used(int K, int slices) {
  const int steps = (K + 31) / 32;
  if (slices <= 1) return 1;
  const int per = (steps + slices - 1) / slices;
  return (steps + per - 1) / per;
}
void launch_bias_act(float* Z, const float* bias, int M, int N, uint16_t* H, int act, hipStream_t s);
void launch_gelu_back(const float* dH, const float* Z, int64_t n, uint16_t* dZ, float* dZf, hipStream_t s);
void launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s);
void launch_head_loss(const float* Y, const float* T, int P, float wt, float* dY, uint16_t* dYb, float* rowloss,
                      hipStream_t s);
void launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, uint16_t* wb, hipStream_t s);
void launch_head_pose(const float* Y, const double* fr_src, const double* fr_tgt, int P, double* R0, double* t0,
                      hipStream_t s);
void launch_head_target(const double* R, const double* t, const double* fr_src, const double* fr_tgt, int P, float* T,
                        hipStream_t s);

}  // namespace hgmm
