// Soft multi-path registration E-step (Sec. 4.1, logarithmic search with
// pruning), gfx950.
//
// A point's expectation of a node is the product of its posteriors among the
// siblings along the path from the root.  Every branch whose expectation is
// at least tau is followed (depth first, an explicit per-lane stack of at
// most 8 entries per level); a branch below tau is pruned with its subtree.
// A followed node that stops by the rule of Algorithm 1 (complexity <=
// lambda_c, no live children, or the last level) receives the point with
// weight E: bins {E, E (T(p) - mu) (3), E, E d_M^2}.  Posteriors come from the
// FP32 scores (exp2 of score differences); offsets and Mahalanobis distances
// at the stop nodes are FP64.  Levels 0-1 are binned in FP64 LDS and added to
// the node bins once per block, deeper nodes with FP64 atomics.

#include "hgmm_dev.h"
#include "hgmm_host.h"

namespace hgmm {

namespace {

__device__ __forceinline__ int64_t level_offset(int l) {
  // (8^(l+1) - 8) / 7
  int64_t p = 8, o = 0;
  for (int i = 0; i < l; ++i) { o += p; p *= 8; }
  return o;
}

constexpr int kBinnedNodes = 72;  // levels 0 and 1 of one tree, binned in LDS

}  // namespace


constexpr int kSoftStack = 8 * 7;  // 8 children per level, up to 6 levels (and one spare level)

__global__ __launch_bounds__(256) void soft_estep_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                         const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                         const TreeDev* __restrict__ trees,
                                                         const NodeF* __restrict__ tab,
                                                         const NodeD* __restrict__ nodes,
                                                         const PoseState* __restrict__ st, double* bins,
                                                         float tau, int32_t* stops_out,
                                                         const int* __restrict__ perm) {
  const Tile tl = tiles[blockIdx.x];
  const int pair = tl.job;
  if (st[pair].done) return;
  const TreeDev& T = trees[pair];
  const int L = T.levels;
  const int64_t nb = T.node_base;
  const int nl = L >= 2 ? kBinnedNodes : 8;
  __shared__ double lbin[kBinnedNodes * 6];
  for (int i = threadIdx.x; i < kBinnedNodes * 6; i += blockDim.x) lbin[i] = 0.0;
  __syncthreads();
  const double R0 = st[pair].R[0], R1 = st[pair].R[1], R2 = st[pair].R[2], R3 = st[pair].R[3],
               R4 = st[pair].R[4], R5 = st[pair].R[5], R6 = st[pair].R[6], R7 = st[pair].R[7],
               R8 = st[pair].R[8], t0 = st[pair].t[0], t1 = st[pair].t[1], t2 = st[pair].t[2];
  for (int b0 = tl.start; b0 < tl.end; b0 += blockDim.x) {
    const int i = b0 + threadIdx.x;
    if (i >= tl.end) continue;
    const double z0 = xs[i], z1 = ys[i], z2 = zs[i];
    const double p0 = R0 * z0 + R1 * z1 + R2 * z2 + t0;
    const double p1 = R3 * z0 + R4 * z1 + R5 * z2 + t1;
    const double p2 = R6 * z0 + R7 * z1 + R8 * z2 + t2;
    int sg[kSoftStack];
    float se[kSoftStack];
    int top = 0, ns = 0;
    int64_t parent = -1;  // local id of the node being expanded (-1: the root's children)
    int plev = -1;
    float pe = 1.0f;
    for (;;) {
      const int cl = plev + 1;
      const int64_t base = level_offset(cl) + (parent < 0 ? 0 : 8 * (parent - level_offset(plev)));
      const NodeF* C = tab + nb + base;
      float s[8];
      float smax = -INFINITY;
      uint32_t lm = 0u;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool on = (C[k].flags & F_LIVE) != 0u;
        float q, m;
        const float sk = score32(C[k], p0, p1, p2, q, m);
        s[k] = on ? sk : -INFINITY;
        lm |= on ? (1u << k) : 0u;
        smax = on ? fmaxf(smax, sk) : smax;
      }
      float den = 0.f;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (lm >> k & 1u) den += __builtin_amdgcn_exp2f(s[k] - smax);
      const float scale = pe / den;
      // pushed in reverse so that the lowest child is expanded first
      for (int k = 7; k >= 0; --k) {
        if (!(lm >> k & 1u)) continue;
        const float e = scale * __builtin_amdgcn_exp2f(s[k] - smax);
        if (e >= tau && top < kSoftStack) {
          sg[top] = (int)(base + k);
          se[top] = e;
          ++top;
        }
      }
      bool expanded = false;
      while (top > 0) {
        --top;
        const int g = sg[top];
        const float e = se[top];
        int l = 0;
        while (level_offset(l + 1) <= g) ++l;
        const uint32_t f = tab[nb + g].flags;
        const bool stop = (f & F_STOP) || !(f & F_HASCH) || (l == L - 1);
        if (!stop) {
          parent = g;
          plev = l;
          pe = e;
          expanded = true;
          break;
        }
        const NodeD& nd = nodes[nb + g];
        const double d0 = p0 - nd.mu[0], d1 = p1 - nd.mu[1], d2 = p2 - nd.mu[2];
        const double w0 = nd.winv[0] * d0;
        const double w1 = nd.winv[1] * d0 + nd.winv[2] * d1;
        const double w2 = nd.winv[3] * d0 + nd.winv[4] * d1 + nd.winv[5] * d2;
        const double m2 = w0 * w0 + w1 * w1 + w2 * w2;
        const double ed = (double)e;
        double* B = (g < nl) ? lbin + g * 6 : bins + (nb + g) * 6;
        unsafeAtomicAdd(B + 0, ed);
        unsafeAtomicAdd(B + 1, ed * d0);
        unsafeAtomicAdd(B + 2, ed * d1);
        unsafeAtomicAdd(B + 3, ed * d2);
        unsafeAtomicAdd(B + 4, ed);
        unsafeAtomicAdd(B + 5, ed * m2);
        ++ns;
      }
      if (!expanded) break;
    }
    if (stops_out) stops_out[perm ? perm[i] : i] = ns;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nl * 6; r += blockDim.x) {
    const int node = r / 6;
    if (lbin[node * 6 + 4] > 0.0) unsafeAtomicAdd(bins + (nb + node) * 6 + (r - node * 6), lbin[r]);
  }
}

void launch_soft_estep(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                       const TreeDev* trees, const NodeF* tab, const NodeD* nodes, const PoseState* st, double* bins,
                       float tau, int32_t* stops_out, const int* perm, hipStream_t s) {
  hipLaunchKernelGGL(soft_estep_kernel, dim3(ntiles), dim3(256), 0, s, xs, ys, zs, tiles, trees, tab, nodes, st, bins,
                     tau, stops_out, perm);
}

}  // namespace hgmm
