// C ABI of the learned warm start: network handle, forward, training step,
// features and the 6D head.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/hgmm.h"
#include "hgmm_dev.h"
#include "hgmm_internal.h"
#include "hgmm_warm.h"

using namespace hgmm;

static const int kDims[5] = {1280, 512, 512, 512, 9};
constexpr int kGradSlices = 8;  // most slices of a GEMM reduction (weight gradients; forward of small batches)

struct hgmm_mlp_s {
  float* w[4] = {};     // FP32 master weights [in x out]
  float* b[4] = {};
  uint16_t* wb[4] = {}; // bf16 copies used by the GEMMs
  float* mw[4] = {};
  float* vw[4] = {};
  float* mb[4] = {};
  float* vb[4] = {};
  float* gw[4] = {};
  float* gb[4] = {};
  int64_t step = 0;
  int cap = 0;          // activation buffers sized for this many rows
  uint16_t* X = nullptr;
  float* Z[4] = {};
  uint16_t* H[4] = {};  // H[l]: bf16 input of layer l (P x kDims[l]); H[0] unused (X)
  float* dH = nullptr;
  float* dZf = nullptr;
  uint16_t* dZb = nullptr;
  float* dY = nullptr;
  uint16_t* dYb = nullptr;
  float* gpart = nullptr;   // partial weight gradients of the reduction slices
  float* rowloss = nullptr;
  float* h_loss = nullptr;  // pinned
};

static int64_t wsize(int l) { return (int64_t)kDims[l] * kDims[l + 1]; }

template <typename T>
static int dalloc(T*& p, int64_t n) {
  if (hipMalloc((void**)&p, sizeof(T) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess)
    return hgmm_fail(HGMM_ENOMEM, "device allocation failed");
  return HGMM_OK;
}

// (frees at teardown: their errors are not reported)
static void mlp_free_acts(hgmm_mlp_s* m) {
  (void)hipFree(m->X);
  for (int l = 0; l < 4; ++l) {
    (void)hipFree(m->Z[l]);
    (void)hipFree(m->H[l]);
    m->Z[l] = nullptr;
    m->H[l] = nullptr;
  }
  (void)hipFree(m->dH);
  (void)hipFree(m->dZf);
  (void)hipFree(m->dZb);
  (void)hipFree(m->dY);
  (void)hipFree(m->dYb);
  (void)hipFree(m->rowloss);
  (void)hipFree(m->gpart);
  if (m->h_loss) (void)hipHostFree(m->h_loss);
  m->X = nullptr; m->dH = nullptr; m->dZf = nullptr; m->dZb = nullptr; m->dY = nullptr; m->dYb = nullptr;
  m->rowloss = nullptr; m->h_loss = nullptr; m->gpart = nullptr;
  m->cap = 0;
}

static int mlp_reserve(hgmm_mlp_s* m, int P) {
  if (P <= m->cap) return HGMM_OK;
  mlp_free_acts(m);
  int rc = 0;
  rc |= dalloc(m->X, (int64_t)P * 1280);
  // Z[l] is the pre-activation output of layer l (P x kDims[l+1]); H[l] is
  // the bf16 input of layer l (P x kDims[l]), H[0] unused (the input is X)
  for (int l = 0; l < 4; ++l) {
    rc |= dalloc(m->Z[l], (int64_t)P * kDims[l + 1]);
    if (l > 0) rc |= dalloc(m->H[l], (int64_t)P * kDims[l]);
  }
  rc |= dalloc(m->dH, (int64_t)P * 512);
  rc |= dalloc(m->dZf, (int64_t)P * 512);
  rc |= dalloc(m->dZb, (int64_t)P * 512);
  rc |= dalloc(m->dY, (int64_t)P * 9);
  rc |= dalloc(m->dYb, (int64_t)P * 9);
  rc |= dalloc(m->rowloss, P);
  rc |= dalloc(m->gpart, (int64_t)kGradSlices * 1280 * 512);
  if (hipHostMalloc((void**)&m->h_loss, sizeof(float) * (size_t)P, hipHostMallocDefault) != hipSuccess) rc = 1;
  if (rc) { mlp_free_acts(m); return hgmm_fail(HGMM_ENOMEM, "activation allocation failed"); }
  m->cap = P;
  return HGMM_OK;
}

// forward from m->X (bf16, P rows); Z[3] holds the 9 outputs.  A small
// batch gives a layer few 64 x 64 output tiles, so its reduction over the
// inputs is split into slices (at least 4 steps of 32 each) until the grid has
// about 128 blocks; the slices' partial products are added in slice order.
static void mlp_forward_core(hgmm_mlp_s* m, int P, hipStream_t s) {
  const uint16_t* in = m->X;
  for (int l = 0; l < 4; ++l) {
    const int K = kDims[l], N = kDims[l + 1];
    const int tiles = ((P + 63) / 64) * ((N + 63) / 64);
    int slices = std::min(kGradSlices, std::max(1, std::min(128 / std::max(tiles, 1), K / 128)));
    while (slices > 1 && (int64_t)slices * P * N > (int64_t)kGradSlices * 1280 * 512) --slices;
    if (slices > 1) {
      launch_gemm_slices(false, false, P, N, K, in, K, m->wb[l], N, m->gpart, N, 0.f, slices, s);
      launch_sum_slices(m->gpart, gemm_slices_used(K, slices), (int64_t)P * N, m->Z[l], s);
    } else {
      launch_gemm(false, false, P, N, K, in, K, m->wb[l], N, m->Z[l], N, 0.f, s);
    }
    launch_bias_act(m->Z[l], m->b[l], P, N, l < 3 ? m->H[l + 1] : nullptr, l < 3 ? 1 : 0, s);
    in = m->H[l + 1];
  }
}

// backward of the loss against targets T (P x 9) into gw/gb; returns via rowloss
static void mlp_backward_core(hgmm_mlp_s* m, const float* T, int P, float wt, hipStream_t s) {
  launch_head_loss(m->Z[3], T, P, wt, m->dY, m->dYb, m->rowloss, s);
  // layer 4 (no activation): dZ4 = dY
  const uint16_t* dZ = m->dYb;
  const float* dZf = m->dY;
  for (int l = 3; l >= 0; --l) {
    const int K = kDims[l], N = kDims[l + 1];
    const uint16_t* Hin = (l == 0) ? m->X : m->H[l];
    // gW = Hin^T dZ  [K x N]: a reduction over the P rows, split into up
    // to kGradSlices parts of at least 512 rows whose partial products are
    // added in slice order
    const int slices = std::min(kGradSlices, std::max(1, P / 512));
    if (slices > 1) {
      launch_gemm_slices(true, false, K, N, P, Hin, K, dZ, N, m->gpart, N, 0.f, slices, s);
      launch_sum_slices(m->gpart, gemm_slices_used(P, slices), (int64_t)K * N, m->gw[l], s);
    } else {
      launch_gemm(true, false, K, N, P, Hin, K, dZ, N, m->gw[l], N, 0.f, s);
    }
    launch_colsum(dZf, P, N, m->gb[l], s);
    if (l == 0) break;
    // dH = dZ W^T [P x K], then through GELU of layer l-1
    launch_gemm(false, true, P, K, N, dZ, N, m->wb[l], N, m->dH, K, 0.f, s);
    launch_gelu_back(m->dH, m->Z[l - 1], (int64_t)P * K, m->dZb, m->dZf, s);
    dZ = m->dZb;
    dZf = m->dZf;
  }
}

extern "C" {

int64_t hgmm_mlp_param_count(void) {
  int64_t n = 0;
  for (int l = 0; l < 4; ++l) n += wsize(l) + kDims[l + 1];
  return n;
}

void hgmm_mlp_destroy(hgmm_mlp m) {
  if (!m) return;
  mlp_free_acts(m);
  for (int l = 0; l < 4; ++l) {
    void* bufs[] = {m->w[l], m->b[l], m->wb[l], m->mw[l], m->vw[l], m->mb[l], m->vb[l], m->gw[l], m->gb[l]};
    for (void* p : bufs) (void)hipFree(p);
  }
  delete m;
}

int hgmm_mlp_set_params(hgmm_mlp m, const float* host) {
  if (!m || !host) return hgmm_fail(HGMM_EINVAL, "null argument");
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    if (hipMemcpy(m->w[l], host + o, sizeof(float) * wsize(l), hipMemcpyHostToDevice) != hipSuccess)
      return hgmm_fail(HGMM_EHIP, "copy failed");
    o += wsize(l);
    if (hipMemcpy(m->b[l], host + o, sizeof(float) * kDims[l + 1], hipMemcpyHostToDevice) != hipSuccess)
      return hgmm_fail(HGMM_EHIP, "copy failed");
    o += kDims[l + 1];
    launch_f32_to_bf16(m->w[l], m->wb[l], wsize(l), nullptr);
  }
  if (hipDeviceSynchronize() != hipSuccess) return hgmm_fail(HGMM_EHIP, "sync failed");
  return HGMM_OK;
}

int hgmm_mlp_get_params(hgmm_mlp m, float* host) {
  if (!m || !host) return hgmm_fail(HGMM_EINVAL, "null argument");
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    if (hipMemcpy(host + o, m->w[l], sizeof(float) * wsize(l), hipMemcpyDeviceToHost) != hipSuccess)
      return hgmm_fail(HGMM_EHIP, "copy failed");
    o += wsize(l);
    if (hipMemcpy(host + o, m->b[l], sizeof(float) * kDims[l + 1], hipMemcpyDeviceToHost) != hipSuccess)
      return hgmm_fail(HGMM_EHIP, "copy failed");
    o += kDims[l + 1];
  }
  return HGMM_OK;
}

int hgmm_mlp_create(uint64_t seed, hgmm_mlp* out) {
  if (!out) return hgmm_fail(HGMM_EINVAL, "null argument");
  hgmm_mlp_s* m = new hgmm_mlp_s();
  int rc = 0;
  for (int l = 0; l < 4; ++l) {
    rc |= dalloc(m->w[l], wsize(l)); rc |= dalloc(m->b[l], kDims[l + 1]); rc |= dalloc(m->wb[l], wsize(l));
    rc |= dalloc(m->mw[l], wsize(l)); rc |= dalloc(m->vw[l], wsize(l)); rc |= dalloc(m->mb[l], kDims[l + 1]);
    rc |= dalloc(m->vb[l], kDims[l + 1]); rc |= dalloc(m->gw[l], wsize(l)); rc |= dalloc(m->gb[l], kDims[l + 1]);
  }
  if (rc) { hgmm_mlp_destroy(m); return hgmm_fail(HGMM_ENOMEM, "parameter allocation failed"); }
  // He-normal weights (std sqrt(2 / fan_in); the head sqrt(1 / fan_in)), zero biases, zero Adam moments
  std::mt19937_64 gen(seed);
  std::vector<float> host((size_t)hgmm_mlp_param_count());
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    std::normal_distribution<double> nd(0.0, std::sqrt((l < 3 ? 2.0 : 1.0) / kDims[l]));
    for (int64_t i = 0; i < wsize(l); ++i) host[o++] = (float)nd(gen);
    for (int i = 0; i < kDims[l + 1]; ++i) host[o++] = 0.f;
  }
  for (int l = 0; l < 4; ++l) {
    if (hipMemset(m->mw[l], 0, sizeof(float) * wsize(l)) != hipSuccess ||
        hipMemset(m->vw[l], 0, sizeof(float) * wsize(l)) != hipSuccess ||
        hipMemset(m->mb[l], 0, sizeof(float) * kDims[l + 1]) != hipSuccess ||
        hipMemset(m->vb[l], 0, sizeof(float) * kDims[l + 1]) != hipSuccess) {
      hgmm_mlp_destroy(m);
      return hgmm_fail(HGMM_EHIP, "clearing the optimiser state failed");
    }
  }
  if ((rc = hgmm_mlp_set_params(m, host.data()))) { hgmm_mlp_destroy(m); return rc; }
  *out = m;
  return HGMM_OK;
}

int hgmm_mlp_forward(hgmm_mlp m, const float* d_X, int P, float* d_Y, void* stream) {
  if (!m || !d_X || !d_Y || P < 1) return hgmm_fail(HGMM_EINVAL, "bad argument");
  int rc = mlp_reserve(m, P);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  launch_f32_to_bf16(d_X, m->X, (int64_t)P * 1280, s);
  mlp_forward_core(m, P, s);
  if (hipMemcpyAsync(d_Y, m->Z[3], sizeof(float) * 9 * P, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return hgmm_fail(HGMM_EHIP, "copy failed");
  if (hipGetLastError() != hipSuccess) return hgmm_fail(HGMM_EHIP, "kernel launch failed");
  return HGMM_OK;
}

static int loss_to_host(hgmm_mlp_s* m, int P, hipStream_t s, double* loss) {
  if (!loss) return HGMM_OK;
  if (hipMemcpyAsync(m->h_loss, m->rowloss, sizeof(float) * P, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return hgmm_fail(HGMM_EHIP, "loss readback failed");
  double t = 0.0;
  for (int i = 0; i < P; ++i) t += m->h_loss[i];
  *loss = t / P;
  return HGMM_OK;
}

int hgmm_mlp_backward(hgmm_mlp m, const float* d_X, const float* d_T, int P, float trans_weight, void* stream,
                      float* host_grads, double* loss) {
  if (!m || !d_X || !d_T || P < 1) return hgmm_fail(HGMM_EINVAL, "bad argument");
  int rc = mlp_reserve(m, P);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  launch_f32_to_bf16(d_X, m->X, (int64_t)P * 1280, s);
  mlp_forward_core(m, P, s);
  mlp_backward_core(m, d_T, P, trans_weight, s);
  if (hipGetLastError() != hipSuccess) return hgmm_fail(HGMM_EHIP, "kernel launch failed");
  if ((rc = loss_to_host(m, P, s, loss))) return rc;
  if (host_grads) {
    if (hipStreamSynchronize(s) != hipSuccess) return hgmm_fail(HGMM_EHIP, "sync failed");
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) {
      if (hipMemcpy(host_grads + o, m->gw[l], sizeof(float) * wsize(l), hipMemcpyDeviceToHost) != hipSuccess)
        return hgmm_fail(HGMM_EHIP, "gradient copy failed");
      o += wsize(l);
      if (hipMemcpy(host_grads + o, m->gb[l], sizeof(float) * kDims[l + 1], hipMemcpyDeviceToHost) != hipSuccess)
        return hgmm_fail(HGMM_EHIP, "gradient copy failed");
      o += kDims[l + 1];
    }
  }
  return HGMM_OK;
}

int hgmm_mlp_train_step(hgmm_mlp m, const float* d_X, const float* d_T, int P, float lr, float trans_weight,
                        void* stream, double* loss) {
  if (!m || !d_X || !d_T || P < 1 || !(lr > 0.f)) return hgmm_fail(HGMM_EINVAL, "bad argument");
  int rc = mlp_reserve(m, P);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  launch_f32_to_bf16(d_X, m->X, (int64_t)P * 1280, s);
  mlp_forward_core(m, P, s);
  mlp_backward_core(m, d_T, P, trans_weight, s);
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float bc1 = 1.f - std::pow(b1, (float)m->step), bc2 = 1.f - std::pow(b2, (float)m->step);
  for (int l = 0; l < 4; ++l) {
    launch_adam(m->w[l], m->mw[l], m->vw[l], m->gw[l], wsize(l), lr, b1, b2, eps, bc1, bc2, m->wb[l], s);
    launch_adam(m->b[l], m->mb[l], m->vb[l], m->gb[l], kDims[l + 1], lr, b1, b2, eps, bc1, bc2, nullptr, s);
  }
  if (hipGetLastError() != hipSuccess) return hgmm_fail(HGMM_EHIP, "kernel launch failed");
  return loss_to_host(m, P, s, loss);
}

int hgmm_warm_features(hgmm_tree forest, const int32_t* h_tree_ids, int n, double reg_eps, float* d_feat,
                       double* d_frames, void* stream) {
  if (!forest || !h_tree_ids || n < 1 || !d_feat || !d_frames) return hgmm_fail(HGMM_EINVAL, "bad argument");
  const int ntrees = hgmm_forest_size(forest);
  for (int i = 0; i < n; ++i)
    if (h_tree_ids[i] < 0 || h_tree_ids[i] >= ntrees) return hgmm_fail(HGMM_EINVAL, "tree id out of range");
  hipStream_t s = (hipStream_t)stream;
  int* d_ids = nullptr;
  if (hipMallocAsync((void**)&d_ids, sizeof(int) * n, s) != hipSuccess) return hgmm_fail(HGMM_ENOMEM, "alloc failed");
  const bool copied = hipMemcpyAsync(d_ids, h_tree_ids, sizeof(int) * n, hipMemcpyHostToDevice, s) == hipSuccess;
  if (copied)
    launch_features(d_ids, n, hgmm_forest_trees(forest), hgmm_forest_nodes(forest), reg_eps, d_feat, d_frames, s);
  const bool freed = hipFreeAsync(d_ids, s) == hipSuccess;
  if (!copied || !freed || hipStreamSynchronize(s) != hipSuccess) return hgmm_fail(HGMM_EHIP, "features failed");
  return HGMM_OK;
}

int hgmm_warm_head_pose(const float* d_Y, const double* d_fr_src, const double* d_fr_tgt, int P, double* d_R0,
                        double* d_t0, void* stream) {
  if (!d_Y || !d_fr_src || !d_fr_tgt || P < 1 || !d_R0 || !d_t0) return hgmm_fail(HGMM_EINVAL, "bad argument");
  launch_head_pose(d_Y, d_fr_src, d_fr_tgt, P, d_R0, d_t0, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return hgmm_fail(HGMM_EHIP, "kernel launch failed");
  return HGMM_OK;
}

int hgmm_warm_head_target(const double* d_R, const double* d_t, const double* d_fr_src, const double* d_fr_tgt,
                          int P, float* d_T, void* stream) {
  if (!d_R || !d_t || !d_fr_src || !d_fr_tgt || P < 1 || !d_T) return hgmm_fail(HGMM_EINVAL, "bad argument");
  launch_head_target(d_R, d_t, d_fr_src, d_fr_tgt, P, d_T, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return hgmm_fail(HGMM_EHIP, "kernel launch failed");
  return HGMM_OK;
}

int hgmm_gemm_bf16(int ta, int tb, int M, int N, int K, const uint16_t* d_A, int lda, const uint16_t* d_B, int ldb,
                   float* d_C, int ldc, void* stream) {
  if (!d_A || !d_B || !d_C || M < 1 || N < 1 || K < 1) return hgmm_fail(HGMM_EINVAL, "bad argument");
  launch_gemm(ta != 0, tb != 0, M, N, K, d_A, lda, d_B, ldb, d_C, ldc, 0.f, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return hgmm_fail(HGMM_EHIP, "kernel launch failed");
  return HGMM_OK;
}

}  // extern "C"
