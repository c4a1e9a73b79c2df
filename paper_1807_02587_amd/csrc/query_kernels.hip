// Point queries against a built tree (gfx950): the log density of each point
// under the model at the node the adaptive descent (Algorithm 1) stops at,
// for consumers of the tree other than registration (scoring a scan against a
// map for loop closure, occupancy queries; the paper names such reuse among
// the benefits of the model, Sec. 6).

#include "hgmm_dev.h"
#include "hgmm_host.h"

namespace hgmm {

// log pi^g - log|cov| / 2 - d_M^2 / 2 - 3/2 log 2 pi of the point T(z) at its
// stop node (local id stop[i] in tree `T`), FP64; -inf for an unassigned point.
__global__ void point_loglik_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                    const float* __restrict__ zs, int64_t n, const int32_t* __restrict__ stop,
                                    const TreeDev* __restrict__ trees, const NodeD* __restrict__ nodes,
                                    const PoseState* __restrict__ st, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t g = stop[i];
  if (g < 0) {
    out[i] = -INFINITY;
    return;
  }
  const PoseState& S = st[0];
  const double z0 = xs[i], z1 = ys[i], z2 = zs[i];
  const double p0 = S.R[0] * z0 + S.R[1] * z1 + S.R[2] * z2 + S.t[0];
  const double p1 = S.R[3] * z0 + S.R[4] * z1 + S.R[5] * z2 + S.t[1];
  const double p2 = S.R[6] * z0 + S.R[7] * z1 + S.R[8] * z2 + S.t[2];
  const NodeD& nd = nodes[trees[0].node_base + g];
  const double d0 = p0 - nd.mu[0], d1 = p1 - nd.mu[1], d2 = p2 - nd.mu[2];
  const double w0 = nd.winv[0] * d0;
  const double w1 = nd.winv[1] * d0 + nd.winv[2] * d1;
  const double w2 = nd.winv[3] * d0 + nd.winv[4] * d1 + nd.winv[5] * d2;
  out[i] = (float)(log(nd.pig) - 0.5 * nd.logdet - 0.5 * (w0 * w0 + w1 * w1 + w2 * w2) - 1.5 * kLog2Pi);
}

void launch_point_loglik(const float* xs, const float* ys, const float* zs, int64_t n, const int32_t* stop,
                         const TreeDev* trees, const NodeD* nodes, const PoseState* st, float* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(point_loglik_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xs, ys, zs, n, stop,
                     trees, nodes, st, out);
}

}  // namespace hgmm
