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
// at the stop nodes are FP64.  Levels 0-1 are staged and binned in LDS (FP64
// bins added to the node bins once per block), deeper nodes are read from the
// records.  Whether a pushed node stops is decided when it is pushed, from
// the flags its parent's scoring read.  Each lane takes one action per step
// (expand a node or bin one stop node); a step's stop nodes are summed across
// the wave per distinct node (FP32 DPP sums of E, E d, E d_M^2) and added with
// one FP64 atomic per value and node.

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


constexpr int kSoftPoints = 128;  // points per block, one per thread

// Stack entry: node id << 4 | stop << 3 | level, with the node's expectation.
__device__ __forceinline__ int soft_pack(int g, bool stop, int l) { return (g << 4) | (stop ? 8 : 0) | l; }

// Grid (tiles, sub-blocks): block (x, y) takes the kSoftPoints points of tile
// x from tl.start + kSoftPoints y.  The scoring records of levels 0-1 (FP32
// and the FP64 prefix) are staged in LDS, and so are the lanes' stacks
// (dynamic LDS of 8 L entries per lane, entry j of thread t at j * kSoftPoints
// + t; a depth-first walk never holds more than 8 entries per level).
__global__ __launch_bounds__(kSoftPoints) void soft_estep_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                         const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                         const TreeDev* __restrict__ trees,
                                                         const NodeF* __restrict__ tab,
                                                         const NodeD* __restrict__ nodes,
                                                         const PoseState* __restrict__ st, double* bins,
                                                         float tau, int32_t* stops_out,
                                                         const int* __restrict__ perm) {
  const Tile tl = tiles[blockIdx.x];
  const int start = tl.start + (int)blockIdx.y * kSoftPoints;
  if (start >= tl.end) return;
  const int pair = tl.job;
  if (st[pair].done) return;
  const int end = tl.end - start < kSoftPoints ? tl.end : start + kSoftPoints;
  const TreeDev& T = trees[pair];
  const int L = T.levels;
  const int64_t nb = T.node_base;
  const int nl = L >= 2 ? kBinnedNodes : 8;
  __shared__ NodeF lf[kBinnedNodes];
  __shared__ NodeS ls[kBinnedNodes];
  __shared__ double lbin[kBinnedNodes * 6];
  for (int r = threadIdx.x; r < nl; r += blockDim.x) {
    const float4* src = reinterpret_cast<const float4*>(&tab[nb + r]);
    float4* dst = reinterpret_cast<float4*>(&lf[r]);
    dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3];
    const NodeD& nd = nodes[nb + r];
    for (int k = 0; k < 3; ++k) ls[r].mu[k] = nd.mu[k];
    for (int k = 0; k < 6; ++k) ls[r].winv[k] = nd.winv[k];
    ls[r].c = nd.c;
  }
  for (int r = threadIdx.x; r < kBinnedNodes * 6; r += blockDim.x) lbin[r] = 0.0;
  __syncthreads();
  const int i = start + (int)threadIdx.x;
  const bool valid = i < end;
  const int lane = __lane_id();
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  if (valid) {
    const PoseState& S = st[pair];
    const double z0 = xs[i], z1 = ys[i], z2 = zs[i];
    p0 = S.R[0] * z0 + S.R[1] * z1 + S.R[2] * z2 + S.t[0];
    p1 = S.R[3] * z0 + S.R[4] * z1 + S.R[5] * z2 + S.t[1];
    p2 = S.R[6] * z0 + S.R[7] * z1 + S.R[8] * z2 + S.t[2];
  }
  extern __shared__ int2 sstk[];
  const int cap = 8 * L;
  int2* stk = sstk + threadIdx.x;
  int top = 0, ns = 0;
  int parent = -1;  // local id of the node to expand (-1: the root's children)
  int plev = -1;
  float pe = 1.0f;
  bool expand = valid, active = valid;
  // one action per lane and step (expand a node, or take one stop node off
  // the stack), so that the stop nodes of a step can be aggregated across the
  // wave before they are binned: lanes of a wave mostly stop at the same node
  while (__ballot(active)) {
    int eg = -1;
    float ee = 0.f, ed0 = 0.f, ed1 = 0.f, ed2 = 0.f, em2 = 0.f;
    if (active) {
      if (expand) {
        const int cl = plev + 1;
        const int base = (int)level_offset(cl) + (parent < 0 ? 0 : 8 * (parent - (int)level_offset(plev)));
        const NodeF* C = (base < nl) ? lf + base : tab + nb + base;
        float sc[8];
        float smax = -INFINITY;
        uint32_t lm = 0u, sm = 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t f = C[k].flags;
          const bool on = (f & F_LIVE) != 0u;
          float q, m;
          const float sk = score32(C[k], p0, p1, p2, q, m);
          sc[k] = on ? sk : -INFINITY;
          lm |= on ? (1u << k) : 0u;
          sm |= ((f & F_STOP) || !(f & F_HASCH) || cl == L - 1) ? (1u << k) : 0u;
          smax = on ? fmaxf(smax, sk) : smax;
        }
        float den = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (lm >> k & 1u) den += __builtin_amdgcn_exp2f(sc[k] - smax);
        const float scale = pe / den;
        // pushed in reverse so that the lowest child is taken first
#pragma unroll
        for (int k = 7; k >= 0; --k) {
          const float e = scale * __builtin_amdgcn_exp2f(sc[k] - smax);
          if ((lm >> k & 1u) && e >= tau && top < cap) {
            stk[top * kSoftPoints] = make_int2(soft_pack(base + k, (sm >> k) & 1u, cl), __float_as_int(e));
            ++top;
          }
        }
        expand = false;
      } else if (top > 0) {
        --top;
        const int2 en = stk[top * kSoftPoints];
        const int ent = en.x;
        const float e = __int_as_float(en.y);
        const int g = ent >> 4;
        if (!(ent & 8)) {
          parent = g;
          plev = ent & 7;
          pe = e;
          expand = true;
        } else {
          const double* mu = (g < nl) ? ls[g].mu : nodes[nb + g].mu;
          const double* wi = (g < nl) ? ls[g].winv : nodes[nb + g].winv;
          const double d0 = p0 - mu[0], d1 = p1 - mu[1], d2 = p2 - mu[2];
          const double w0 = wi[0] * d0;
          const double w1 = wi[1] * d0 + wi[2] * d1;
          const double w2 = wi[3] * d0 + wi[4] * d1 + wi[5] * d2;
          eg = g;
          ee = e;
          ed0 = (float)((double)e * d0);
          ed1 = (float)((double)e * d1);
          ed2 = (float)((double)e * d2);
          em2 = (float)((double)e * (w0 * w0 + w1 * w1 + w2 * w2));
          ++ns;
        }
      } else {
        active = false;
      }
    }
    // this step's stop nodes: equal nodes summed across the wave, one add each
    bool pend = eg >= 0;
    unsigned long long pending = __ballot(pend);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int key = __shfl(eg, leader, 64);
      const bool mine = pend && (eg == key);
      const unsigned long long mm = __ballot(mine);
      const float v0 = wave_sum(mine ? ee : 0.f);
      const float v1 = wave_sum(mine ? ed0 : 0.f);
      const float v2 = wave_sum(mine ? ed1 : 0.f);
      const float v3 = wave_sum(mine ? ed2 : 0.f);
      const float v5 = wave_sum(mine ? em2 : 0.f);
      if (lane == leader) {
        double* B = (key < nl) ? lbin + key * 6 : bins + (nb + key) * 6;
        unsafeAtomicAdd(B + 0, (double)v0);
        unsafeAtomicAdd(B + 1, (double)v1);
        unsafeAtomicAdd(B + 2, (double)v2);
        unsafeAtomicAdd(B + 3, (double)v3);
        unsafeAtomicAdd(B + 4, (double)v0);
        unsafeAtomicAdd(B + 5, (double)v5);
      }
      pend = pend && !mine;
      pending &= ~mm;
    }
  }
  if (valid && stops_out) stops_out[perm ? perm[i] : i] = ns;
  __syncthreads();
  for (int r = threadIdx.x; r < nl * 6; r += blockDim.x) {
    const int node = r / 6;
    if (lbin[node * 6 + 4] > 0.0) unsafeAtomicAdd(bins + (nb + node) * 6 + (r - node * 6), lbin[r]);
  }
}

void launch_soft_estep(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                       int tile_points, int max_levels, const TreeDev* trees, const NodeF* tab, const NodeD* nodes,
                       const PoseState* st, double* bins, float tau, int32_t* stops_out, const int* perm,
                       hipStream_t s) {
  const unsigned nsub = (unsigned)((tile_points + kSoftPoints - 1) / kSoftPoints);
  // the deepest tree of the call sets the stack: 8 entries per level
  const size_t lds = sizeof(int2) * (size_t)kSoftPoints * 8 * (size_t)max_levels;
  hipLaunchKernelGGL(soft_estep_kernel, dim3(ntiles, nsub), dim3(kSoftPoints), lds, s, xs, ys, zs, tiles, trees, tab,
                     nodes, st, bins, tau, stops_out, perm);
}

}  // namespace hgmm
