// GMM-Tree registration kernels (gfx950).
//
// E-step (Sec. 4.1, Algorithm 1): every point of the moving cloud is
// transformed in FP64, then descends the tree along the most likely child
// (8 FP64 Mahalanobis scores per level) until the chosen node is simple
// enough (complexity <= lambda_c), has no live children, or is on the last
// level.  The point's weight at that node is its posterior among the siblings
// of the last level visited.  Per-node moments are summed over runs of equal
// stop nodes inside a wavefront and added in fixed point, through a
// block-shared table in LDS, to the node bins in HBM.
// M-step (Sec. 4.2, Eq. 8-16): one 1024-thread block per pair reads and
// clears the node bins, lets every node with mass contribute weighted
// point-to-plane rows along its three eigen-directions to the 6x6 normal
// equations, solves them by Cholesky and applies the exact rotation of the
// solved angle vector.
#include "hgmm_dev.h"
#include "hgmm_host.h"

namespace hgmm {

__device__ __forceinline__ int64_t lvl_off(int l) {
  // (8^(l+1) - 8) / 7
  int64_t p = 8;
  int64_t o = 0;
  for (int i = 0; i < l; ++i) { o += p; p *= 8; }
  return o;
}

__global__ void set_stop_flags_kernel(NodeF* tab, const NodeD* __restrict__ nodes, int64_t n, double lambda_c) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  uint32_t f = tab[g].flags & ~F_STOP;
  if ((f & F_LIVE) && nodes[g].kappa <= lambda_c) f |= F_STOP;
  tab[g].flags = f;
}

// The descent's FP64 scoring records (NodeR) with this call's stop flags.  A
// dead node gets mu = 0, W = 0 and c = -inf, so that scoring 8 children
// needs no liveness test.
__global__ void reg_table_kernel(const NodeF* __restrict__ tab, const NodeD* __restrict__ nodes, NodeR* rt, int64_t n,
                                 double lambda_c) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const uint32_t f = tab[g].flags;
  NodeR r;
  if (f & F_LIVE) {
    const NodeD& nd = nodes[g];
    for (int i = 0; i < 3; ++i) r.mu[i] = nd.mu[i];
    for (int i = 0; i < 6; ++i) r.w[i] = nd.winv[i] * kWScale;
    r.c = nd.c * kLog2e;
    r.flags = (f & ~F_STOP) | (nd.kappa <= lambda_c ? F_STOP : 0u);
  } else {
    for (int i = 0; i < 3; ++i) r.mu[i] = 0.0;
    for (int i = 0; i < 6; ++i) r.w[i] = 0.0;
    r.c = -INFINITY;
    r.flags = 0u;
  }
  r.pad[0] = r.pad[1] = r.pad[2] = 0u;
  rt[g] = r;
}

// Initial transform of every pair: rows of `stride` doubles (stride 0 = the
// same transform for all pairs).
__global__ void init_pose_kernel(PoseState* st, int npairs, const double* __restrict__ R0, const double* __restrict__ t0,
                                 int stride, const int* __restrict__ active) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= npairs) return;
  PoseState& S = st[b];
  const double* R = R0 + (size_t)stride * b;
  const double* t = t0 + (size_t)stride * b;
  for (int i = 0; i < 9; ++i) S.R[i] = R[i];
  for (int i = 0; i < 3; ++i) S.t[i] = t[i];
  for (int i = 0; i < 6; ++i) S.x[i] = 0.0;
  S.loglik = 0.0;
  S.iters = 0;
  S.done = (active && !active[b]) ? 1 : 0;
  S.status = 0;
}

// The most likely child among the 8 descent records at C, in FP64 (dead
// children score -inf, so there is no liveness test; the lowest index wins
// an exact tie).  Returns the child, -1 when none is live, and leaves every
// child's score in s and the winner's in s1.
template <typename RecPtr>
__device__ __forceinline__ int choose_child64(RecPtr C, double p0, double p1, double p2, double (&s)[8],
                                              double& s1) {
#pragma unroll
  for (int k = 0; k < 8; ++k) s[k] = C[k].c - quad_r(C[k], p0, p1, p2);
  int k1 = -1;
  s1 = -INFINITY;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (s[k] > s1) { s1 = s[k]; k1 = k; }
  return k1;
}

constexpr int kLdsNodes = 72;    // levels 0 and 1 of one tree
constexpr double kTwoLn2 = 1.3862943611198906;  // 2 / log2(e)

// Runs of equal keys inside the 16-lane rows of a wave.  A run starts at
// the first lane of a row or where the key differs from the previous lane's.
// Returns the first lane of this lane's run and sets `end` on the run's last
// lane.  All 64 lanes must be active.
__device__ __forceinline__ int row_run(int key, int lane, bool& end) {
  // the previous lane's key in the row (row_shr:1); the row's first lane
  // keeps key ^ 1, so it always starts a run
  const int prev = __builtin_amdgcn_update_dpp(key ^ 1, key, 0x111, 0xF, 0xF, false);
  const unsigned long long heads = __ballot(prev != key);
  end = ((lane & 15) == 15) || (((heads >> 1) >> lane) & 1ull);
  return 63 - __clzll((long long)(heads & ((2ull << lane) - 1ull)));
}

// One step of the segmented inclusive sum over the runs of row_run (shift SH
// = 1, 2, 4, 8 in turn): a lane adds the value SH lanes before it when that
// lane is in its run (`take` 1 or 0).  The data flow is fixed, so the run
// sums do not depend on timing.
template <int SH>
__device__ __forceinline__ void run_step(float (&v)[kFixVals], float take) {
#pragma unroll
  for (int j = 0; j < kFixVals; ++j) v[j] = fmaf(dpp_f<0x110 + SH>(v[j]), take, v[j]);
}

// Block-shared fixed-point bins in LDS: bin k of the first kLdsNodes is node
// k of levels 0-1; the others are keyed by node (open addressing with linear
// probing; a bin's pad word holds its node + 1, 0 when free).  124 bins
// (11.6 KB) keep the descent's LDS at 26.4 KB, six blocks of four waves per
// compute unit.
constexpr int kHashSlots = 124;
constexpr int kHashProbes = 16;

// The keyed bin of `key` (a node below levels 0-1), claimed when free; -1
// when the probes find none (the caller then adds to the node bin in HBM).
__device__ __forceinline__ int hash_slot(FixBin* tab, int key) {
  constexpr int kKeyed = kHashSlots - kLdsNodes;
  const unsigned long long tag = (unsigned long long)key + 1ull;
  int slot = kLdsNodes + (int)(((((unsigned)key * 0x9E3779B1u) >> 24) * (unsigned)kKeyed) >> 8);
  for (int p = 0; p < kHashProbes; ++p) {
    const unsigned long long prev = atomicCAS(&tab[slot].pad, 0ull, tag);
    if (prev == 0ull || prev == tag) return slot;
    slot = slot + 1 == kHashSlots ? kLdsNodes : slot + 1;
  }
  return -1;
}

// A run of equal stop nodes staged for its adds: its bin (-1: none, add to
// the node bin in HBM), node (local id), number of points and the sums
// {M0, D (3), Q}.
struct WaveRun {
  int slot;
  int key;
  unsigned n;
  float v[kFixVals];
};

// Orders one wave's LDS writes before its later LDS reads of other lanes'
// values (a wave's LDS operations complete in order; this keeps the compiler
// from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One E-step over the tiles of every pair (tiles[].job is the pair index).
// Each point is transformed in FP64 and descends the tree (Algorithm 1); the
// posterior weight at its stop node is formed once per wave after the
// descent, from the stop level's scores that each lane keeps.
// Moments: neighbouring lanes of a wave with the same stop node form runs,
// summed in FP32 by a fixed-order segmented scan inside each 16-lane row and
// carried across row boundaries; each run's sums and count are added in
// fixed point (FixBin) to the block's bin of its node in LDS (one bin per
// node of levels 0-1, deeper nodes in bins keyed by node), and at the end of
// the block six neighbouring
// lanes per node add each table bin to the node bin in HBM (when the table is
// full a run goes to the node bin directly).  Fixed-point sums are integers,
// whose totals do not depend on the order of the adds, so the moments, and
// the registration, are bitwise reproducible.
// Scores are FP64 (full rate on CDNA4, as FP32 without packing), so the
// chosen child is the FP64 argmax and the weight needs no rounding bound.
// NLEV: number of leading tree levels whose scoring records are staged in
// LDS (2: the 72 nodes of levels 0-1, 7 KB; 3: also the 512 of level 2).
// Grid: 8 * per_xcd blocks.  Consecutive blocks are dispatched to consecutive
// XCDs, so block b takes tile (b % 8) * per_xcd + b / 8: every XCD works
// through one contiguous range of tiles (of pairs), whose node records then
// stay in that XCD's L2.
// work (nullable, profiling): adds the points processed and the levels they
// scored to work[0] and work[1].  Held to 6 waves per SIMD (at most 80
// VGPRs), which the LDS allows, for latency hiding; with level 2 staged
// (74 KB of LDS) two blocks fit on a compute unit.
// rtab: the descent's FP64 scoring records (reg_table_kernel).
// ATOMICS: the comparison mode, in which the run sums are added to FP64 node
// bins (bins, 6 values per node, every level) with FP64 atomics instead.
template <int NLEV, bool ATOMICS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NLEV >= 3 ? 2 : 6))) void descend_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                      const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                      int ntiles, int per_xcd, const TreeDev* __restrict__ trees,
                                                      const NodeR* __restrict__ rtab,
                                                      const PoseState* __restrict__ st, FixBin* fbins,
                                                      double* bins, int32_t* stop_out, float* gamma_out,
                                                      const int* __restrict__ perm, int max_levels,
                                                      unsigned long long* work) {
  const int tix = (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3);
  if (tix >= ntiles) return;
  const Tile tl = tiles[tix];
  const int pair = tl.job;
  if (st[pair].done) return;
  const TreeDev& T = trees[pair];
  // levels the descent may use (a cap acts like a tree built with fewer levels)
  const int L = (max_levels > 0 && max_levels < T.levels) ? max_levels : T.levels;
  const int64_t nb = T.node_base;
  constexpr int kStaged = NLEV >= 3 ? 584 : kLdsNodes;
  __shared__ NodeR lds[kStaged];
  __shared__ FixBin hbin[kHashSlots];
  __shared__ WaveRun wrun[4][64];
  __shared__ unsigned long long wsum[2];
  const int nst = L >= NLEV ? kStaged : (L >= 2 ? 72 : 8);
  {
    constexpr int kWords = (int)(sizeof(NodeR) / sizeof(float4));
    const float4* src = reinterpret_cast<const float4*>(rtab + nb);
    float4* dst = reinterpret_cast<float4*>(lds);
    for (int i = threadIdx.x; i < nst * kWords; i += blockDim.x) dst[i] = src[i];
  }
  {
    unsigned long long* z = &hbin[0].lo[0];
    for (int i = threadIdx.x; i < kHashSlots * (int)(sizeof(FixBin) / 8); i += blockDim.x) z[i] = 0ull;
    if (threadIdx.x < 2) wsum[threadIdx.x] = 0ull;
  }
  __syncthreads();
  const double R0 = st[pair].R[0], R1 = st[pair].R[1], R2 = st[pair].R[2], R3 = st[pair].R[3],
               R4 = st[pair].R[4], R5 = st[pair].R[5], R6 = st[pair].R[6], R7 = st[pair].R[7],
               R8 = st[pair].R[8], t0 = st[pair].t[0], t1 = st[pair].t[1], t2 = st[pair].t[2];
  const int lane = __lane_id();
  const int wv = threadIdx.x >> 6;
  const double sD = kFixScaleD / (T.extent > 0.0 ? T.extent : 1.0);
  unsigned my_points = 0u, my_levels = 0u;
  for (int b0 = tl.start; b0 < tl.end; b0 += blockDim.x) {
    const int i = b0 + threadIdx.x;
    const bool valid = i < tl.end;
    int64_t g = -1;
    float gam = 0.f, d0 = 0.f, d1 = 0.f, d2 = 0.f, dm2 = 0.f;
    if (valid) {
      const double z0 = xs[i], z1 = ys[i], z2 = zs[i];
      const double p0 = R0 * z0 + R1 * z1 + R2 * z2 + t0;
      const double p1 = R3 * z0 + R4 * z1 + R5 * z2 + t1;
      const double p2 = R6 * z0 + R7 * z1 + R8 * z2 + t2;
      int parent = 0;
      int l = 0;
      // the stop level's child scores stay in these registers while other
      // lanes of the wave descend further
      double s[8], sk = 0.0;
      int kst = -1;
      int64_t lbst = 0;
      // one level: false when the descent ends here (no live child, or the
      // chosen child is the stop node).  Each call site passes its own kind
      // of pointer, so the records are read with scalar loads, LDS reads or
      // vector loads as that site's address allows.
      auto level = [&](const NodeR* C, int64_t lbase) -> bool {
        const int k = choose_child64(C, p0, p1, p2, s, sk);
        if (k < 0) return false;  // no live node here: the point is left unassigned
        const uint32_t flags = C[k].flags;
        if ((flags & F_STOP) || !(flags & F_HASCH) || (l == L - 1)) {
          kst = k;
          lbst = lbase;
          return false;
        }
        parent = 8 * parent + k;
        return true;
      };
      bool go = true;
      while (go && l < L) {
        const int64_t lbase = lvl_off(l) + 8 * (int64_t)parent;
        // the lanes still descending are all at level l.  When they also
        // share the parent (always at level 0, and mostly below it, as the
        // points are in Morton order), its 8 records are read once for the
        // wave with scalar loads and the FP64 arithmetic takes them from
        // scalar registers; otherwise each lane reads them, from the LDS
        // copy for the staged levels.
        const int lu = __builtin_amdgcn_readfirstlane(l);
        const int pu = __builtin_amdgcn_readfirstlane(parent);
        if (__ballot(parent != pu) == 0ull) go = level(rtab + nb + lvl_off(lu) + 8 * (int64_t)pu, lbase);
        else if (l < NLEV) go = level(lds + lbase, lbase);
        else go = level(rtab + nb + lbase, lbase);
        if (go) ++l;
      }
      my_points += 1u;
      my_levels += (unsigned)min(l + 1, L);
      if (kst >= 0) {
        // weight of the point at the chosen node: its posterior among the
        // live siblings, gamma = 1 / sum_j 2^(s_j - s_k) (dead siblings add
        // 2^-inf = 0).  The FP64 differences rounded to FP32 and the FP32
        // exp2 and sum keep gamma within 1e-6 relative.
        float den = 1.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) den += (j == kst) ? 0.f : __builtin_amdgcn_exp2f((float)(s[j] - sk));
        gam = 1.0f / den;
        g = nb + lbst + kst;
        // offset from the node mean (one FP32 rounding of an FP64 difference)
        // and the squared Mahalanobis distance in FP64
        auto offset = [&](const NodeR& nr) {
          d0 = (float)(p0 - nr.mu[0]);
          d1 = (float)(p1 - nr.mu[1]);
          d2 = (float)(p2 - nr.mu[2]);
          dm2 = (float)(quad_r(nr, p0, p1, p2) * kTwoLn2);
        };
        if (g - nb < nst) offset(lds[g - nb]);
        else offset(rtab[g]);
      }
      const int oi = perm ? perm[i] : i;
      if (stop_out) stop_out[oi] = g >= 0 ? (int32_t)(g - nb) : -1;
      if (gamma_out) gamma_out[oi] = gam;
    }
    // run sums of {gamma, gamma d (3), d^2} over equal stop nodes in each row
    // (an unassigned point has key -1 and zero sums)
    const int key = g >= 0 ? (int)(g - nb) : -1;
    float v[kFixVals] = {gam, gam * d0, gam * d1, gam * d2, dm2};
    bool run_end;
    const int rs = row_run(key, lane, run_end);
    run_step<1>(v, lane - 1 >= rs ? 1.f : 0.f);
    run_step<2>(v, lane - 2 >= rs ? 1.f : 0.f);
    run_step<4>(v, lane - 4 >= rs ? 1.f : 0.f);
    run_step<8>(v, lane - 8 >= rs ? 1.f : 0.f);
    // a run that goes on across a row boundary: the boundary lane hands its
    // sums to the lanes of the next row whose run starts at that row's first
    // lane (rows in order, so a run over several rows collects all of them),
    // and only the run's last lane adds
    int rw = rs;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int bl = 16 * r + 15;
      if (__builtin_amdgcn_readlane(key, bl) == __builtin_amdgcn_readlane(key, bl + 1)) {
        const int sb = __builtin_amdgcn_readlane(rw, bl);
        const bool cont = rw == bl + 1;
#pragma unroll
        for (int j = 0; j < kFixVals; ++j) {
          const float vb = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v[j]), bl));
          v[j] += cont ? vb : 0.f;
        }
        rw = cont ? sb : rw;
        run_end = run_end && lane != bl;
      }
    }
    // the runs' sums to their nodes' bins in the block's table: the last lane
    // of each run claims the bin and stages the run in the wave's LDS rows,
    // then six neighbouring lanes take one run each (five sums and the
    // count), so the conversions to fixed point and the adds spread over
    // the wave
    const bool emit = run_end && key >= 0;
    const unsigned long long ends = __ballot(emit);
    if (ends != 0ull) {
      wave_lds_sync();  // the previous points' reads of the rows are done
      if (emit) {
        WaveRun& w = wrun[wv][__popcll(ends & ((1ull << lane) - 1ull))];
        w.slot = ATOMICS ? -1 : key < kLdsNodes ? key : hash_slot(hbin, key);
        w.key = key;
        w.n = (unsigned)(lane - rw + 1);
#pragma unroll
        for (int j = 0; j < kFixVals; ++j) w.v[j] = v[j];
      }
      wave_lds_sync();
      const int nruns = __popcll(ends);
      for (int r0 = 0; r0 < nruns; r0 += 10) {
        const int r = r0 + lane / 6, col = lane - 6 * (lane / 6);
        if (lane >= 60 || r >= nruns) continue;
        const WaveRun& w = wrun[wv][r];
        const int k = w.key, sl = w.slot;
        if (ATOMICS) {
          // bins order {M0, D, count, Q}
          unsafeAtomicAdd(bins + (nb + k) * 6 + (col < 4 ? col : 9 - col), col == 5 ? (double)w.n : (double)w.v[col]);
        } else if (col == 5) {
          if (sl >= 0) atomicAdd(&hbin[sl].cnt, (unsigned long long)w.n);
          else atomicAdd(&fbins[nb + k].cnt, (unsigned long long)w.n);
        } else {
          unsigned long long lo;
          long long hi;
          fix_split((double)w.v[col] * (col == 0 ? kFixScaleM0 : col < 4 ? sD : kFixScaleQ), lo, hi);
          if (sl >= 0) fix_add(&hbin[sl].lo[col], &hbin[sl].hi[col], lo, hi);
          else fix_add(&fbins[nb + k].lo[col], &fbins[nb + k].hi[col], lo, hi);
        }
      }
    }
  }
  __syncthreads();
  // the table's bins into the node bins in HBM: six neighbouring lanes per
  // bin (five sums and the count), so one atomic instruction adds to a few
  // whole bins
  for (int t = threadIdx.x; !ATOMICS && t < kHashSlots * 6; t += blockDim.x) {
    const int slot = t / 6, col = t - 6 * slot;
    if (hbin[slot].cnt == 0ull) continue;
    FixBin& G = fbins[nb + (slot < kLdsNodes ? (int64_t)slot : (int64_t)(hbin[slot].pad - 1ull))];
    if (col == 5) atomicAdd(&G.cnt, hbin[slot].cnt);
    else fix_add(&G.lo[col], &G.hi[col], hbin[slot].lo[col], hbin[slot].hi[col]);
  }
  if (work) {
    atomicAdd(&wsum[0], (unsigned long long)my_points);
    atomicAdd(&wsum[1], (unsigned long long)my_levels);
    __syncthreads();
    if (threadIdx.x == 0) {
      atomicAdd(&work[0], wsum[0]);
      atomicAdd(&work[1], wsum[1]);
    }
  }
}

// The node bins of the fixed-point moments as FP64 bins {M0, D (3), count,
// Q} (for callers that read the bins directly).  One block per pair.
__global__ __launch_bounds__(256) void fold_bins_kernel(const TreeDev* __restrict__ trees,
                                                        const FixBin* __restrict__ fbins, double* bins) {
  const TreeDev& T = trees[blockIdx.x];
  const int64_t nn = lvl_off(T.levels);
  for (int64_t g = T.node_base + threadIdx.x; g < T.node_base + nn; g += blockDim.x) {
    double b[6];
    fix_read(fbins[g], T.extent, b);
    double* B = bins + g * 6;
    for (int j = 0; j < 6; ++j) B[j] = b[j];
  }
}

// ---------------------------------------------------------------------------
// Single-level E-step ("GMM J=n", Sec. 5 list of variants)
// ---------------------------------------------------------------------------
//
// The live nodes of one tree level form a mixture of J = 8^(level+1)
// components with their global weights.  Every point is scored against every
// component (a linear scan instead of the tree's logarithmic descent), in
// FP64, keeping the maximum (lowest index on exact ties) and the denominator
// sum_j 2^(s_j - m) against a reference score m that moves only when a score
// exceeds it by more than kFlatLag.  A move multiplies the old sum by less
// than 2^-kFlatLag, so the FP32 exp2 of each term and of the rescale keep
// the posterior within 1e-6 relative.  Every lane of a wave scores the same
// component at a time, so the components' records are read with scalar
// loads.  The moments go to the node bins with FP64 atomics after
// aggregation of equal components inside a wave.  The tree's records carry
// the weight inside the sibling group; the single-level mixture needs the
// global weight, so the E-step reads records rebuilt with it
// (flat_table_kernel).

// The FP64 scoring records of every node with the global weight pi^g in the
// constant: c = log2(e) (log pi^g - log|cov| / 2), W = sqrt(log2(e) / 2) L^-1.
// A dead component gets mu = 0, W = 0 and c = -inf, so it scores -inf for
// every point and adds nothing to the running sums: the scan has no liveness
// test.
__global__ void flat_table_kernel(const NodeF* __restrict__ tab, const NodeD* __restrict__ nodes, NodeR* fr,
                                  int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const NodeD& nd = nodes[g];
  NodeR r;
  if ((tab[g].flags & F_LIVE) && nd.pig > 0.0) {
    for (int k = 0; k < 3; ++k) r.mu[k] = nd.mu[k];
    for (int k = 0; k < 6; ++k) r.w[k] = nd.winv[k] * kWScale;
    r.c = (log(nd.pig) - 0.5 * nd.logdet) * kLog2e;
    r.flags = F_LIVE;
  } else {
    for (int k = 0; k < 3; ++k) r.mu[k] = 0.0;
    for (int k = 0; k < 6; ++k) r.w[k] = 0.0;
    r.c = -INFINITY;
    r.flags = 0u;
  }
  r.pad[0] = r.pad[1] = r.pad[2] = 0u;
  fr[g] = r;
}

// a component record read through the constant address space: the kernel
// never writes the table, so reads at a wave-uniform address are scalar loads
typedef const __attribute__((address_space(4))) NodeR ConstNodeR;

constexpr int kFlatSlices = 4;      // waves per block; wave w scans slice w of the components
constexpr double kFlatLag = 8.0;    // the reference score moves when a score exceeds it by more

// Running state of a scan over components for one point: the maximum s1 and
// its index k1, the reference m (s1 - kFlatLag <= m <= s1) and
// den = sum_j 2^(s_j - m).
struct FlatState {
  double s1, m, den;
  int k1;
};

__device__ __forceinline__ void flat_init(FlatState& a) {
  a.s1 = -INFINITY;
  a.m = -INFINITY;
  a.den = 0.0;
  a.k1 = -1;
}

__device__ __forceinline__ void flat_add(FlatState& a, double s, int j) {
  const bool up = s > a.s1;  // strict: the lower index stays on equal scores
  a.k1 = up ? j : a.k1;
  a.s1 = up ? s : a.s1;
  const bool live = s > -INFINITY;
  const double d = s - a.m;  // +inf before the first live component
  const bool move = live && !(d <= kFlatLag);
  const double e = (double)__builtin_amdgcn_exp2f((float)(move ? -d : d));
  a.den = move ? fma(a.den, e, 1.0) : (live ? a.den + e : a.den);
  a.m = move ? s : a.m;
}

// a <- a merged with b, where b holds components of higher index than a
__device__ __forceinline__ void flat_merge(FlatState& a, const FlatState& b) {
  const bool up = b.s1 > a.s1;
  a.k1 = up ? b.k1 : a.k1;
  a.s1 = up ? b.s1 : a.s1;
  const double m = fmax(a.m, b.m);
  const double ra = a.m > -INFINITY ? (double)__builtin_amdgcn_exp2f((float)(a.m - m)) : 0.0;
  const double rb = b.m > -INFINITY ? (double)__builtin_amdgcn_exp2f((float)(b.m - m)) : 0.0;
  a.den = fma(a.den, ra, b.den * rb);
  a.m = m;
}

// Grid (tiles, sub-blocks): block (x, y) takes the 64 P points of tile x from
// tl.start + 64 P y.  Its 4 waves each scan a quarter of the components for
// all of those points (P per lane), reading the records with scalar loads;
// the four partial states are merged in LDS in component order, and the
// first 64 P threads finish one point each.
template <int P>
__global__ __launch_bounds__(256) void flat_estep_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                         const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                         const TreeDev* __restrict__ trees,
                                                         const NodeR* __restrict__ ftab,
                                                         const PoseState* __restrict__ st, double* bins,
                                                         int32_t* stop_out, float* gamma_out,
                                                         const int* __restrict__ perm, int level) {
  constexpr int NP = 64 * P;
  const Tile tl = tiles[blockIdx.x];
  const int start = tl.start + (int)blockIdx.y * NP;
  if (start >= tl.end) return;
  const int pair = tl.job;
  if (st[pair].done) return;
  const int end = tl.end - start < NP ? tl.end : start + NP;
  const TreeDev& T = trees[pair];
  const int64_t nb = T.node_base;
  const int64_t g0 = nb + lvl_off(level);
  const int J = 8 << (3 * level);
  const NodeR* __restrict__ Fg = ftab + g0;
  const double R0 = st[pair].R[0], R1 = st[pair].R[1], R2 = st[pair].R[2], R3 = st[pair].R[3],
               R4 = st[pair].R[4], R5 = st[pair].R[5], R6 = st[pair].R[6], R7 = st[pair].R[7],
               R8 = st[pair].R[8], t0 = st[pair].t[0], t1 = st[pair].t[1], t2 = st[pair].t[2];
  const int lane = __lane_id();
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double px[P], py[P], pz[P];
  FlatState S[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int i = start + lane + 64 * q;
    const bool v = i < end;
    const double z0 = v ? (double)xs[i] : 0.0, z1 = v ? (double)ys[i] : 0.0, z2 = v ? (double)zs[i] : 0.0;
    px[q] = R0 * z0 + R1 * z1 + R2 * z2 + t0;
    py[q] = R3 * z0 + R4 * z1 + R5 * z2 + t1;
    pz[q] = R6 * z0 + R7 * z1 + R8 * z2 + t2;
    flat_init(S[q]);
  }
  const int per = J / kFlatSlices;
  const int jb = wv * per;
  const ConstNodeR* Cg = (const ConstNodeR*)(Fg + jb);
#pragma unroll 2
  for (int jj = 0; jj < per; ++jj) {
    const ConstNodeR& C = Cg[jj];
#pragma unroll
    for (int q = 0; q < P; ++q) flat_add(S[q], C.c - quad_r(C, px[q], py[q], pz[q]), jb + jj);
  }
  __shared__ double ms[kFlatSlices][3][NP];
  __shared__ int mk[kFlatSlices][NP];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int r = lane + 64 * q;
    ms[wv][0][r] = S[q].s1;
    ms[wv][1][r] = S[q].m;
    ms[wv][2][r] = S[q].den;
    mk[wv][r] = S[q].k1;
  }
  __syncthreads();
  const int r = (int)threadIdx.x;
  if (r >= NP) return;  // whole waves leave; no barrier follows
  FlatState A;
  A.s1 = ms[0][0][r]; A.m = ms[0][1][r]; A.den = ms[0][2][r]; A.k1 = mk[0][r];
#pragma unroll
  for (int w = 1; w < kFlatSlices; ++w) {
    FlatState B;
    B.s1 = ms[w][0][r]; B.m = ms[w][1][r]; B.den = ms[w][2][r]; B.k1 = mk[w][r];
    flat_merge(A, B);
  }
  const int i = start + r;
  const bool valid = i < end;
  int64_t g = -1;
  float gam = 0.f, d0 = 0.f, d1 = 0.f, d2 = 0.f, dm2 = 0.f;
  if (valid && A.k1 >= 0) {
    const double z0 = xs[i], z1 = ys[i], z2 = zs[i];
    const double p0 = R0 * z0 + R1 * z1 + R2 * z2 + t0;
    const double p1 = R3 * z0 + R4 * z1 + R5 * z2 + t1;
    const double p2 = R6 * z0 + R7 * z1 + R8 * z2 + t2;
    // the winner's share: 2^(s1 - m) / den, 0 <= s1 - m <= kFlatLag
    gam = (float)((double)__builtin_amdgcn_exp2f((float)(A.s1 - A.m)) / A.den);
    g = g0 + A.k1;
    const NodeR& nd = Fg[A.k1];
    d0 = (float)(p0 - nd.mu[0]);
    d1 = (float)(p1 - nd.mu[1]);
    d2 = (float)(p2 - nd.mu[2]);
    dm2 = (float)(quad_r(nd, p0, p1, p2) * kTwoLn2);
  }
  if (valid) {
    const int oi = perm ? perm[i] : i;
    if (stop_out) stop_out[oi] = g >= 0 ? (int32_t)(g - nb) : -1;
    if (gamma_out) gamma_out[oi] = gam;
  }
  // aggregate equal components inside the wave, then one FP64 atomic add each
  bool pend = valid && g >= 0;
  unsigned long long pending = __ballot(pend);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int64_t key = __shfl(g, leader, 64);
    const bool mine = pend && (g == key);
    const unsigned long long mm = __ballot(mine);
    const float v0 = wave_sum(mine ? gam : 0.f);
    const float v1 = wave_sum(mine ? gam * d0 : 0.f);
    const float v2 = wave_sum(mine ? gam * d1 : 0.f);
    const float v3 = wave_sum(mine ? gam * d2 : 0.f);
    const float v5 = wave_sum(mine ? dm2 : 0.f);
    if (lane == leader) {
      double* B = bins + key * 6;
      unsafeAtomicAdd(B + 0, (double)v0);
      unsafeAtomicAdd(B + 1, (double)v1);
      unsafeAtomicAdd(B + 2, (double)v2);
      unsafeAtomicAdd(B + 3, (double)v3);
      unsafeAtomicAdd(B + 4, (double)__popcll(mm));
      unsafeAtomicAdd(B + 5, (double)v5);
    }
    pend = pend && !mine;
    pending &= ~mm;
  }
}

// ---------------------------------------------------------------------------
// M-step
// ---------------------------------------------------------------------------

constexpr int kNormThreads = 1024;  // one block per pair
constexpr int kNV = 28;             // 21 (upper H) + 6 (g) + 1 (log-likelihood numerator)

__device__ inline bool chol6_solve(const double* Hu /*21 upper*/, double shift, const double* g, double* x) {
  double A[6][6];
  int idx = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) { A[i][j] = Hu[idx]; A[j][i] = Hu[idx]; ++idx; }
  double Lm[6][6];
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j] + shift;
    for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
    if (!(d > 0.0)) return false;
    Lm[j][j] = sqrt(d);
    for (int i = j + 1; i < 6; ++i) {
      double v = A[i][j];
      for (int k = 0; k < j; ++k) v -= Lm[i][k] * Lm[j][k];
      Lm[i][j] = v / Lm[j][j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double v = g[i];
    for (int k = 0; k < i; ++k) v -= Lm[i][k] * y[k];
    y[i] = v / Lm[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 6; ++k) v -= Lm[k][i] * x[k];
    x[i] = v / Lm[i][i];
  }
  return true;
}

// Contribution of one node with moments b = {M0, D (3), count, sum d2} to the
// normal equations (Eq. 11-16, increment about the model mean o) and to the
// log-likelihood numerator.
__device__ __forceinline__ void node_terms(const NodeD& nd, const double* b, double N, double o0, double o1, double o2,
                                           double (&acc)[kNV]) {
  const double m0 = b[0];
  const double pis = m0 / N;
  const double dl0 = b[1] / m0, dl1 = b[2] / m0, dl2 = b[3] / m0;
  const double c0 = nd.mu[0] + dl0 - o0, c1 = nd.mu[1] + dl1 - o1, c2 = nd.mu[2] + dl2 - o2;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double n0 = nd.evec[3 * l], n1 = nd.evec[3 * l + 1], n2 = nd.evec[3 * l + 2];
    const double w = pis / nd.lam[l];
    const double a[6] = {c1 * n2 - c2 * n1, c2 * n0 - c0 * n2, c0 * n1 - c1 * n0, n0, n1, n2};
    const double r = n0 * dl0 + n1 * dl1 + n2 * dl2;
    int idx = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
#pragma unroll
      for (int v = u; v < 6; ++v) { acc[idx] += w * a[u] * a[v]; ++idx; }
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) acc[21 + u] -= w * a[u] * r;
  }
  acc[27] += b[4] * (log(nd.pig) - 0.5 * nd.logdet) - 0.5 * b[5];
}

// One block per pair.  mode 0: normal equations from this iteration's moments
// (the descent's fixed-point node bins, read and cleared), Cholesky solve and
// pose update.  mode 1: the same sums from the FP64 bins alone, written to
// out[pair * 28 ..] (H upper, g, mean log-likelihood).  mode 2: as mode 0
// with every node's moments read and cleared from the FP64 bins (the
// single-level and soft E-steps add FP64 moments there).
__global__ __launch_bounds__(kNormThreads) void normal_kernel(double* bins, FixBin* fbins,
                                                              const NodeD* __restrict__ nodes,
                                                              const TreeDev* __restrict__ trees, PoseState* st,
                                                              const int64_t* __restrict__ n_moving, int mode,
                                                              double tol_rot, double tol_trans_rel, int max_iters,
                                                              double* out) {
  const int pair = blockIdx.x;
  PoseState& S = st[pair];
  if (S.done) return;
  const TreeDev& T = trees[pair];
  const int64_t nn = lvl_off(T.levels);
  const int64_t nb = T.node_base;
  const double N = (double)n_moving[pair];
  const double o0 = T.origin[0], o1 = T.origin[1], o2 = T.origin[2];
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  // every node with mass adds its rows to the normal equations
  double acc[kNV];
#pragma unroll
  for (int v = 0; v < kNV; ++v) acc[v] = 0.0;
  for (int64_t g = threadIdx.x; g < nn; g += kNormThreads) {
    double b[6];
    if (mode == 0) {
      FixBin& F = fbins[nb + g];
      if (F.cnt == 0ull) continue;
      fix_read(F, T.extent, b);
#pragma unroll
      for (int j = 0; j < kFixVals; ++j) { F.lo[j] = 0ull; F.hi[j] = 0ll; }
      F.cnt = 0ull;
    } else {
      double* B = bins + (nb + g) * 6;
      b[0] = B[0];
      if (!(b[0] > 0.0)) continue;
      b[1] = B[1]; b[2] = B[2]; b[3] = B[3]; b[4] = B[4]; b[5] = B[5];
      if (mode == 2) { B[0] = 0.0; B[1] = 0.0; B[2] = 0.0; B[3] = 0.0; B[4] = 0.0; B[5] = 0.0; }
    }
    if (b[0] > 0.0) node_terms(nodes[nb + g], b, N, o0, o1, o2, acc);
  }
  __shared__ double red[kNormThreads / 64][kNV];
  __shared__ double tot[kNV];
#pragma unroll
  for (int v = 0; v < kNV; ++v) {
    const double sv = wave_sum_dd(acc[v]);
    if (lane == 0) red[wv][v] = sv;
  }
  __syncthreads();
  if (threadIdx.x < kNV) {
    double sv = 0.0;
    for (int w = 0; w < kNormThreads / 64; ++w) sv += red[w][threadIdx.x];
    tot[threadIdx.x] = sv;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double ll = tot[27] / N - 1.5 * kLog2Pi;
  if (mode == 1) {
    for (int v = 0; v < kNV; ++v) out[pair * kNV + v] = tot[v];
    out[pair * kNV + 27] = ll;
    return;
  }
  S.loglik = ll;
  S.iters += 1;
  double x[6];
  bool ok = chol6_solve(tot, 0.0, tot + 21, x);
  if (!ok) {
    double tr = tot[0] + tot[6] + tot[11] + tot[15] + tot[18] + tot[20];
    ok = (tr > 0.0) && chol6_solve(tot, 1e-12 * tr, tot + 21, x);
  }
  if (!ok) {
    S.status = -6;
    S.done = 1;
    return;
  }
  for (int i = 0; i < 6; ++i) S.x[i] = x[i];
  // exact rotation of the angle vector omega (Rodrigues), composed on the left
  const double w0 = x[0], w1 = x[1], w2 = x[2];
  const double th = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
  double A, Bc;
  if (th < 1e-12) { A = 1.0; Bc = 0.0; }
  else { A = sin(th) / th; Bc = (1.0 - cos(th)) / (th * th); }
  const double K[9] = {0, -w2, w1, w2, 0, -w0, -w1, w0, 0};
  double Ri[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double k2 = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
      Ri[3 * i + j] = (i == j ? 1.0 : 0.0) + A * K[3 * i + j] + Bc * k2;
    }
  double Rn[9], tn[3];
  const double dt0 = S.t[0] - o0, dt1 = S.t[1] - o1, dt2 = S.t[2] - o2;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) Rn[3 * i + j] = Ri[3 * i] * S.R[j] + Ri[3 * i + 1] * S.R[3 + j] + Ri[3 * i + 2] * S.R[6 + j];
    tn[i] = Ri[3 * i] * dt0 + Ri[3 * i + 1] * dt1 + Ri[3 * i + 2] * dt2 + T.origin[i] + x[3 + i];
  }
  for (int i = 0; i < 9; ++i) S.R[i] = Rn[i];
  for (int i = 0; i < 3; ++i) S.t[i] = tn[i];
  const double tau = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
  if ((th < tol_rot && tau < tol_trans_rel * T.extent) || S.iters >= max_iters) S.done = 1;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

void launch_set_stop_flags(NodeF* tab, const NodeD* nodes, int64_t n, double lambda_c, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(set_stop_flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, nodes, n, lambda_c);
}

void launch_init_pose(PoseState* st, int npairs, const double* R0, const double* t0, int stride, const int* active,
                      hipStream_t s) {
  hipLaunchKernelGGL(init_pose_kernel, dim3((npairs + 63) / 64), dim3(64), 0, s, st, npairs, R0, t0, stride, active);
}

// Scoring records of an imported tree.
__global__ void import_nodes_kernel(NodeD* nodes, NodeF* tab, int64_t n) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  NodeD& a = nodes[g];
  NodeF nf;
  NodeD tmp;
  uint32_t flags = 0u;
  if (a.live && make_node(a.mu, a.cov, a.pi, tmp, nf)) {
    for (int i = 0; i < 6; ++i) a.winv[i] = tmp.winv[i];
    a.c = tmp.c;
    a.logdet = tmp.logdet;
    flags = F_LIVE | (a.has_children ? F_HASCH : 0u);
  } else {
    a.live = 0;
    nf = NodeF{};
  }
  nf.flags = flags;
  tab[g] = nf;
}

void launch_import_nodes(NodeD* nodes, NodeF* tab, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(import_nodes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nodes, tab, n);
}

void launch_reg_table(const NodeF* tab, const NodeD* nodes, NodeR* rt, int64_t n, double lambda_c, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(reg_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, nodes, rt, n, lambda_c);
}

void launch_descend(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                    const TreeDev* trees, const NodeR* rtab, const PoseState* st, FixBin* fbins,
                    double* atomic_bins, int32_t* stop_out, float* gamma_out, const int* perm, int lds_levels,
                    int max_levels, unsigned long long* work, hipStream_t s) {
  if (ntiles <= 0) return;
  const int per_xcd = (ntiles + 7) / 8;
  const dim3 grid((unsigned)(8 * per_xcd));
#define HGMM_DESCEND(NL, AT)                                                                                          \
  hipLaunchKernelGGL((descend_kernel<NL, AT>), grid, dim3(256), 0, s, xs, ys, zs, tiles, ntiles, per_xcd, trees, rtab,\
                     st, fbins, atomic_bins, stop_out, gamma_out, perm, max_levels, work)
  if (atomic_bins) {
    if (lds_levels >= 3) HGMM_DESCEND(3, true);
    else HGMM_DESCEND(2, true);
  } else {
    if (lds_levels >= 3) HGMM_DESCEND(3, false);
    else HGMM_DESCEND(2, false);
  }
#undef HGMM_DESCEND
}

void launch_flat_table(const NodeF* tab, const NodeD* nodes, NodeR* fr, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(flat_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, nodes, fr, n);
}

void launch_flat_estep(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                       int tile_points, const TreeDev* trees, const NodeR* ftab, const PoseState* st, double* bins,
                       int32_t* stop_out, float* gamma_out, const int* perm, int level, hipStream_t s) {
  constexpr int P = 1;
  const unsigned nsub = (unsigned)((tile_points + 64 * P - 1) / (64 * P));
  hipLaunchKernelGGL((flat_estep_kernel<P>), dim3(ntiles, nsub), dim3(256), 0, s, xs, ys, zs, tiles, trees, ftab, st,
                     bins, stop_out, gamma_out, perm, level);
}

void launch_fold_bins(const TreeDev* trees, const FixBin* fbins, double* bins, int npairs, hipStream_t s) {
  hipLaunchKernelGGL(fold_bins_kernel, dim3(npairs), dim3(256), 0, s, trees, fbins, bins);
}

void launch_normal(double* bins, FixBin* fbins, const NodeD* nodes, const TreeDev* trees, PoseState* st,
                   const int64_t* n_moving, int npairs, int mode, double tol_rot, double tol_trans_rel, int max_iters,
                   double* out, hipStream_t s) {
  hipLaunchKernelGGL(normal_kernel, dim3(npairs), dim3(kNormThreads), 0, s, bins, fbins, nodes, trees, st, n_moving,
                     mode, tol_rot, tol_trans_rel, max_iters, out);
}

int normal_values() { return kNV; }

}  // namespace hgmm
