// GMM-Tree construction kernels (gfx950).
//
// A level of the tree is fitted for every parent at once.  Points are kept
// sorted by their parent, so each parent owns a contiguous range of the point
// arrays; that range is cut into tiles of one wavefront each.  Per EM
// iteration a tile evaluates the 8 child scores of each of its points
// (Sec. 3, Eq. 2-3), turns them into responsibilities and accumulates the
// responsibility-weighted zeroth, first and second moments of every child
// about the child's current mean (80 FP32 sums per lane).  The sums are
// reduced across the wave with DPP and written as FP64 tile partials; a
// second launch folds each parent's partials in a fixed order and runs the
// FP64 M-step for its 8 children, so no block waits on another and no
// device-scope fence is needed.  Parents with few points run all their EM
// iterations inside one wave instead (em_fused_kernel).
#include "hgmm_dev.h"
#include "hgmm_host.h"

#include <algorithm>
#include <type_traits>

namespace hgmm {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

void launch_fill_u32(void* p, uint32_t v, int64_t n_words, hipStream_t s) {
  if (n_words <= 0) return;
  int64_t blocks = (n_words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, v, n_words);
}

// Work items of a launch: blockIdx.x, blockIdx.x + gridDim.x, ... below n, or
// below *dn when the count lives on the device (a level planned on the device,
// launched with a fixed grid).  With dn null and one block per item this is
// exactly one item per block.
__device__ __forceinline__ int work_count(const int* dn, int n) { return dn ? *dn : n; }

__device__ __forceinline__ void copy_nodef(NodeF& dst, const NodeF& src) {
  const float4* s = reinterpret_cast<const float4*>(&src);
  float4* d = reinterpret_cast<float4*>(&dst);
  d[0] = s[0]; d[1] = s[1]; d[2] = s[2]; d[3] = s[3];
}

// ---------------------------------------------------------------------------
// root statistics (the tile list of level 0 has one job per tree root)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void root_mean_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                       const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                       double* partials, size_t pstride, const int* dn, int n) {
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Tile tl = tiles[w];
  const int lane = threadIdx.x;
  double s0 = 0, s1 = 0, s2 = 0;
  float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
  int bad = 0;
  for (int i = tl.start + lane; i < tl.end; i += 64) {
    float x = xs[i], y = ys[i], z = zs[i];
    bad |= !(isfinite(x) && isfinite(y) && isfinite(z));
    s0 += x; s1 += y; s2 += z;
    lo0 = fminf(lo0, x); lo1 = fminf(lo1, y); lo2 = fminf(lo2, z);
    hi0 = fmaxf(hi0, x); hi1 = fmaxf(hi1, y); hi2 = fmaxf(hi2, z);
  }
  s0 = wave_sum_dd(s0); s1 = wave_sum_dd(s1); s2 = wave_sum_dd(s2);
  for (int m = 32; m >= 1; m >>= 1) {
    lo0 = fminf(lo0, __shfl_xor(lo0, m, 64)); lo1 = fminf(lo1, __shfl_xor(lo1, m, 64));
    lo2 = fminf(lo2, __shfl_xor(lo2, m, 64)); hi0 = fmaxf(hi0, __shfl_xor(hi0, m, 64));
    hi1 = fmaxf(hi1, __shfl_xor(hi1, m, 64)); hi2 = fmaxf(hi2, __shfl_xor(hi2, m, 64));
  }
  bad = __any(bad);
  if (lane == 0) {
    const double vals[10] = {s0, s1, s2, (double)lo0, (double)lo1, (double)lo2, (double)hi0, (double)hi1,
                             (double)hi2, (double)bad};
    for (int v = 0; v < 10; ++v) partials[(size_t)v * pstride + w] = vals[v];
  }
  }
}

// One wave per tree: fixed-order fold of the root-mean tile partials.
__global__ __launch_bounds__(64) void root_mean_fold_kernel(const Job* __restrict__ jobs, TreeDev* trees,
                                                            const double* __restrict__ partials, size_t pstride,
                                                            const int* dn, int n) {
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Job jb = jobs[w];
  const int lane = threadIdx.x;
  double a[3], bb[1];
  wave_fold<3, 8>(partials + jb.tile_first, pstride, jb.ntiles, lane, a);
  wave_fold<1, 8>(partials + 9 * pstride + jb.tile_first, pstride, jb.ntiles, lane, bb);
  const double a0 = a[0], a1 = a[1], a2 = a[2], b = bb[0];
  double l0 = INFINITY, l1 = INFINITY, l2 = INFINITY, h0 = -INFINITY, h1 = -INFINITY, h2 = -INFINITY;
  for (int t = lane; t < jb.ntiles; t += 64) {
    const size_t c = (size_t)jb.tile_first + t;
    l0 = fmin(l0, partials[3 * pstride + c]); l1 = fmin(l1, partials[4 * pstride + c]);
    l2 = fmin(l2, partials[5 * pstride + c]); h0 = fmax(h0, partials[6 * pstride + c]);
    h1 = fmax(h1, partials[7 * pstride + c]); h2 = fmax(h2, partials[8 * pstride + c]);
  }
  for (int m = 32; m >= 1; m >>= 1) {
    l0 = fmin(l0, __shfl_xor(l0, m, 64)); l1 = fmin(l1, __shfl_xor(l1, m, 64));
    l2 = fmin(l2, __shfl_xor(l2, m, 64)); h0 = fmax(h0, __shfl_xor(h0, m, 64));
    h1 = fmax(h1, __shfl_xor(h1, m, 64)); h2 = fmax(h2, __shfl_xor(h2, m, 64));
  }
  if (lane == 0) {
    TreeDev& T = trees[jb.tree];
    double n = (double)jb.count;
    T.origin[0] = a0 / n; T.origin[1] = a1 / n; T.origin[2] = a2 / n;
    T.extent = sqrt((h0 - l0) * (h0 - l0) + (h1 - l1) * (h1 - l1) + (h2 - l2) * (h2 - l2));
    if (b > 0) T.status = -3;
  }
  }
}

__global__ __launch_bounds__(64) void root_cov_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                      const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                      const Job* __restrict__ jobs, const TreeDev* __restrict__ trees,
                                                      double* partials, size_t pstride, const int* dn, int n) {
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Tile tl = tiles[w];
  const Job jb = jobs[tl.job];
  const int lane = threadIdx.x;
  const double o0 = trees[jb.tree].origin[0], o1 = trees[jb.tree].origin[1], o2 = trees[jb.tree].origin[2];
  double c[6] = {0, 0, 0, 0, 0, 0};
  for (int i = tl.start + lane; i < tl.end; i += 64) {
    double d0 = (double)xs[i] - o0, d1 = (double)ys[i] - o1, d2 = (double)zs[i] - o2;
    c[0] += d0 * d0; c[1] += d0 * d1; c[2] += d0 * d2; c[3] += d1 * d1; c[4] += d1 * d2; c[5] += d2 * d2;
  }
  for (int k = 0; k < 6; ++k) c[k] = wave_sum_dd(c[k]);
  if (lane < 6) {
    double v = c[0];
    for (int k = 1; k < 6; ++k) v = (lane == k) ? c[k] : v;
    partials[(size_t)lane * pstride + w] = v;
  }
  }
}

__global__ __launch_bounds__(64) void root_cov_fold_kernel(const Job* __restrict__ jobs, TreeDev* trees,
                                                           const double* __restrict__ partials, size_t pstride,
                                                           double eps, const int* dn, int n) {
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Job jb = jobs[w];
  const int lane = threadIdx.x;
  double a[6];
  wave_fold<6, 8>(partials + jb.tile_first, pstride, jb.ntiles, lane, a);
  if (lane == 0) {
    TreeDev& T = trees[jb.tree];
    double n = (double)jb.count;
    for (int k = 0; k < 6; ++k) T.root_cov[k] = a[k] / n;
    T.root_cov[0] += eps; T.root_cov[3] += eps; T.root_cov[5] += eps;
    eig_sym3(T.root_cov, T.root_lam, T.root_evec);
  }
  }
}

// ---------------------------------------------------------------------------
// PCA-octant initialisation of the children of every job's parent
// ---------------------------------------------------------------------------

__global__ void init_children_kernel(const Job* __restrict__ jobs, int njobs, const TreeDev* __restrict__ trees,
                                     NodeD* nodes, NodeF* tab, double eps, const int* dn) {
  const int nj = work_count(dn, njobs);
  for (int gid = blockIdx.x * blockDim.x + threadIdx.x; gid < 8 * nj; gid += gridDim.x * blockDim.x) {
  const int j = gid >> 3, k = gid & 7;
  const Job jb = jobs[j];
  double pmu[3], plam[3], pev[9];
  if (jb.parent < 0) {
    const TreeDev& T = trees[jb.tree];
    for (int i = 0; i < 3; ++i) { pmu[i] = T.origin[i]; plam[i] = T.root_lam[i]; }
    for (int i = 0; i < 9; ++i) pev[i] = T.root_evec[i];
  } else {
    const NodeD& P = nodes[jb.parent];
    for (int i = 0; i < 3; ++i) { pmu[i] = P.mu[i]; plam[i] = P.lam[i]; }
    for (int i = 0; i < 9; ++i) pev[i] = P.evec[i];
  }
  // child k covers the eigen-octant with sign + on axis a when bit a of k is 0;
  // mean and covariance of a Gaussian restricted to it (half-normal moments)
  const double hn_mean = 0.79788456080286535588;   // sqrt(2/pi)
  const double hn_var = 0.36338022763241865692;    // 1 - 2/pi
  double mu[3] = {pmu[0], pmu[1], pmu[2]};
  double cov[6] = {eps, 0, 0, eps, 0, eps};
  for (int a = 0; a < 3; ++a) {
    double lr = fmax(plam[a] - eps, 0.0);
    double sg = ((k >> a) & 1) ? -1.0 : 1.0;
    double off = sg * hn_mean * sqrt(lr);
    const double* e = pev + 3 * a;
    mu[0] += off * e[0]; mu[1] += off * e[1]; mu[2] += off * e[2];
    double v = hn_var * lr;
    cov[0] += v * e[0] * e[0]; cov[1] += v * e[0] * e[1]; cov[2] += v * e[0] * e[2];
    cov[3] += v * e[1] * e[1]; cov[4] += v * e[1] * e[2]; cov[5] += v * e[2] * e[2];
  }
  const int g = jb.child_base + k;
  NodeD nd;
  NodeF nf;
  NodeD& out = nodes[g];
  if (make_node(mu, cov, 0.125, nd, nf)) {
    for (int i = 0; i < 3; ++i) out.mu[i] = nd.mu[i];
    for (int i = 0; i < 6; ++i) { out.cov[i] = nd.cov[i]; out.winv[i] = nd.winv[i]; }
    out.pi = nd.pi; out.c = nd.c; out.logdet = nd.logdet; out.live = 1;
    copy_nodef(tab[g], nf);
  } else {
    out.live = 0; out.pi = 0.0;
    tab[g].flags = 0u;
  }
  }
}

// ---------------------------------------------------------------------------
// EM: responsibilities and moments of one point against the 8 children
// ---------------------------------------------------------------------------

// Offsets are taken from a reference point of the job (the mean of its first
// live child): each point is brought to FP32 once, q = float(p - ref), and the
// offset from child k is d = q - m_k with m_k = float(mu_k - ref).  This keeps
// FP64 arithmetic out of the per-child work; the extra rounding is a few units
// of the last place of |q| + |m_k|, far below the scale of the covariances.
struct __align__(16) EmFrame {
  float p[8][10];  // per child: mean - reference point [3], scoring rows [6], constant
  double ref[3];
};

// Reference point and FP32 child parameters of a job in its local frame (all
// 64 lanes of a wave call it; lanes 0..7 write their child).  A dead child
// gets offset 0, rows 0 and constant -inf: its score is -inf, so its
// responsibility and moment contributions are exactly 0.  `live` must be
// non-zero.
__device__ __forceinline__ void em_frame(const NodeF* ch, uint32_t live, EmFrame& f, int tid) {
  const int r = __ffs(live) - 1;
  if (tid < 3) f.ref[tid] = ch[r].mu[tid];
  if (tid < 8) {
    const bool on = (live >> tid) & 1u;
    float* q = f.p[tid];
    for (int i = 0; i < 3; ++i) q[i] = on ? (float)(ch[tid].mu[i] - ch[r].mu[i]) : 0.f;
    for (int i = 0; i < 6; ++i) q[3 + i] = on ? ch[tid].w[i] : 0.f;
    q[9] = on ? ch[tid].c : -INFINITY;
  }
}

// Two ways to hand the children's parameters (the same for every lane) to
// the per-point E-step.  ChildParams reads the frame once (20 aligned 16-byte
// LDS reads) into scalar registers, where they stay for all points of the
// iteration: best when a block runs many points per iteration.  FrameParams
// re-reads them from LDS (broadcast reads) for every point: no set-up cost,
// best for a one-iteration tile launch with few points per thread.
struct ChildParams {
  float pm[8][3], pw[8][6], pc[8];
  __device__ float m(int k, int i) const { return pm[k][i]; }
  __device__ float w(int k, int i) const { return pw[k][i]; }
  __device__ float c(int k) const { return pc[k]; }
};

struct FrameParams {
  const EmFrame& f;
  __device__ float m(int k, int i) const { return f.p[k][i]; }
  __device__ float w(int k, int i) const { return f.p[k][3 + i]; }
  __device__ float c(int k) const { return f.p[k][9]; }
};

__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ __forceinline__ void child_params(const EmFrame& f, ChildParams& u) {
  const float4* src = reinterpret_cast<const float4*>(&f.p[0][0]);
  float t[80];
#pragma unroll
  for (int j = 0; j < 20; ++j) {
    const float4 v = src[j];
    t[4 * j] = v.x; t[4 * j + 1] = v.y; t[4 * j + 2] = v.z; t[4 * j + 3] = v.w;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int i = 0; i < 3; ++i) u.pm[k][i] = uniform_f(t[10 * k + i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) u.pw[k][i] = uniform_f(t[10 * k + 3 + i]);
    u.pc[k] = uniform_f(t[10 * k + 9]);
  }
}

// Responsibilities of the 8 children for one point (local frame) and its
// moment contributions (about each child's mean).  Branch-free: dead
// children carry the score -inf (see em_frame), so the scheduler can
// interleave the 8 independent score chains.
template <typename P>
__device__ __forceinline__ void em_point(const P& u, float q0, float q1, float q2, float (&a)[8][10]) {
  float s[8];
  float smax = -INFINITY;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float d0 = q0 - u.m(k, 0), d1 = q1 - u.m(k, 1), d2 = q2 - u.m(k, 2);
    const float w0 = u.w(k, 0) * d0;
    const float w1 = fmaf(u.w(k, 1), d0, u.w(k, 2) * d1);
    const float w2 = fmaf(u.w(k, 3), d0, fmaf(u.w(k, 4), d1, u.w(k, 5) * d2));
    s[k] = u.c(k) - fmaf(w0, w0, fmaf(w1, w1, w2 * w2));
    smax = fmaxf(smax, s[k]);
  }
  float e[8], sum = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = __builtin_amdgcn_exp2f(s[k] - smax);
    sum += e[k];
  }
  const float inv = 1.0f / sum;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float r = e[k] * inv;
    const float d0 = q0 - u.m(k, 0), d1 = q1 - u.m(k, 1), d2 = q2 - u.m(k, 2);
    const float r0 = r * d0, r1 = r * d1, r2 = r * d2;
    a[k][0] += r;
    a[k][1] += r0; a[k][2] += r1; a[k][3] += r2;
    a[k][4] = fmaf(r0, d0, a[k][4]);
    a[k][5] = fmaf(r0, d1, a[k][5]);
    a[k][6] = fmaf(r0, d2, a[k][6]);
    a[k][7] = fmaf(r1, d1, a[k][7]);
    a[k][8] = fmaf(r1, d2, a[k][8]);
    a[k][9] = fmaf(r2, d2, a[k][9]);
  }
}

// Up to KP points of one thread (points first, first + STRIDE, ...) held in
// registers: loaded once with all loads in flight together, then reused (by
// every EM iteration of a block-per-parent job).
template <int KP>
struct PointCache {
  float x[KP], y[KP], z[KP];
};

template <int STRIDE, int KP>
__device__ __forceinline__ void load_points(const float* __restrict__ xs, const float* __restrict__ ys,
                                            const float* __restrict__ zs, int start, int end, int first,
                                            PointCache<KP>& c) {
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int i = start + first + k * STRIDE;
    const bool ok = i < end;
    c.x[k] = ok ? xs[i] : 0.f;
    c.y[k] = ok ? ys[i] : 0.f;
    c.z[k] = ok ? zs[i] : 0.f;
  }
}

// Moments of this thread's points of [start, end): the first KP come from the
// cache, any further ones are streamed with the next point's loads issued
// before the current point's arithmetic.
template <int STRIDE, int KP, bool LDS_PARAMS, typename P>
__device__ __forceinline__ void em_points(const float* __restrict__ xs, const float* __restrict__ ys,
                                          const float* __restrict__ zs, int start, int end, int first,
                                          const PointCache<KP>& c, const P& u, const double (&ref)[3],
                                          float (&a)[8][10]) {
  const double r0 = ref[0], r1 = ref[1], r2 = ref[2];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (start + first + k * STRIDE >= end) break;
    // with LDS parameters, re-read them for every point rather than holding
    // ~80 of them in vector registers across the loop
    if constexpr (LDS_PARAMS) asm volatile("" ::: "memory");
    em_point(u, (float)((double)c.x[k] - r0), (float)((double)c.y[k] - r1), (float)((double)c.z[k] - r2), a);
  }
  int i = start + first + KP * STRIDE;
  if (i >= end) return;
  float nx = xs[i], ny = ys[i], nz = zs[i];
  for (; i < end; i += STRIDE) {
    const float px = nx, py = ny, pz = nz;
    if (i + STRIDE < end) { nx = xs[i + STRIDE]; ny = ys[i + STRIDE]; nz = zs[i + STRIDE]; }
    if constexpr (LDS_PARAMS) asm volatile("" ::: "memory");
    em_point(u, (float)((double)px - r0), (float)((double)py - r1), (float)((double)pz - r2), a);
  }
}

// E-step and moment sums of the points first, first + STRIDE, ... of
// [start, end): the first KP from the register cache, the rest streamed.
// HOIST selects scalar-register (ChildParams) or LDS (FrameParams) parameters.
template <int STRIDE, int KP, bool HOIST>
__device__ __forceinline__ void em_range(const float* __restrict__ xs, const float* __restrict__ ys,
                                         const float* __restrict__ zs, int start, int end, int first,
                                         const PointCache<KP>& c, const EmFrame& f, float (&a)[8][10]) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int v = 0; v < 10; ++v) a[k][v] = 0.f;
  if constexpr (HOIST) {
    ChildParams u;
    child_params(f, u);
    em_points<STRIDE, KP, false>(xs, ys, zs, start, end, first, c, u, f.ref, a);
  } else {
    const FrameParams u{f};
    em_points<STRIDE, KP, true>(xs, ys, zs, start, end, first, c, u, f.ref, a);
  }
}

// One butterfly step of the row reduce-scatter: the first H values are kept
// by the lane whose role is "low", the next H by its partner; each lane adds
// the partner's copy of the half it keeps (DPP pattern CTRL pairs the lanes).
template <int H, int CTRL>
__device__ __forceinline__ void rs_step(float (&a)[8][10], bool hi) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float lo_v = a[i / 10][i % 10], hi_v = a[(i + H) / 10][(i + H) % 10];
    const float keep = hi ? hi_v : lo_v;
    const float send = hi ? lo_v : hi_v;
    a[i / 10][i % 10] = keep + dpp_f<CTRL>(send);
  }
}

// Reduce-scatter of the 80 per-lane sums over each 16-lane row in four
// butterfly steps (row mirror, half-row mirror, quad xor 2, quad xor 1).
// Afterwards lane r of a row holds the row totals of values 5r .. 5r+4 in
// a[0][0..4].  Fixed data flow, so the result does not depend on timing.
__device__ __forceinline__ void row_reduce_scatter80(float (&a)[8][10], int r) {
  rs_step<40, 0x140>(a, r >= 8);
  rs_step<20, 0x141>(a, (r & 7) >= 4);
  rs_step<10, 0x4E>(a, (r & 2) != 0);
  rs_step<5, 0xB1>(a, (r & 1) != 0);
}

// Row totals of all lanes of a block into rows[tid / 16][0..79].
__device__ __forceinline__ void rows_store80(float (&a)[8][10], float (*rows)[80], int tid) {
  row_reduce_scatter80(a, tid & 15);
  float* out = rows[tid >> 4] + 5 * (tid & 15);
#pragma unroll
  for (int j = 0; j < 5; ++j) out[j] = a[0][j];
}

// FP64 M-step of the 8 children of one parent from the 80 combined sums
// (moments about the means the E-step used).  Runs on one full wave; lanes 0..7
// own one child each.  Updates the LDS copy of the children; GLOBAL: also the
// FP32 table and the FP64 node records (the final iteration), else only the
// FP32 scoring records are formed (make_nodef_fast).  FRAME: the same lanes
// also write the next E-step's frame (what em_frame would compute from the
// updated children).
template <bool GLOBAL = true, bool FRAME = false>
__device__ __forceinline__ void mstep_children(const double* tot, NodeF* ch, NodeF* tab, NodeD* nodes,
                                               int child_base, double eps, double min_mass, int lane,
                                               EmFrame* fr = nullptr) {
  // surviving mass of the parent, summed pairwise in the same order on every lane
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double n = tot[k * 10];
    v[k] = ((ch[k].flags & F_LIVE) && n >= min_mass) ? n : 0.0;
  }
  const double total = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  bool live = false;
  double mu[3] = {0.0, 0.0, 0.0};
  NodeF nf;
  if (lane < 8) {
    const int g = child_base + lane;
    const double N = tot[lane * 10];
    live = (ch[lane].flags & F_LIVE) != 0 && N >= min_mass;
    NodeD nd;
    if (live) {
      const double* A = tot + lane * 10;
      const double inv = 1.0 / N;
      const double dl0 = A[1] * inv, dl1 = A[2] * inv, dl2 = A[3] * inv;
      mu[0] = ch[lane].mu[0] + dl0; mu[1] = ch[lane].mu[1] + dl1; mu[2] = ch[lane].mu[2] + dl2;
      double cov[6] = {A[4] * inv - dl0 * dl0 + eps, A[5] * inv - dl0 * dl1, A[6] * inv - dl0 * dl2,
                       A[7] * inv - dl1 * dl1 + eps, A[8] * inv - dl1 * dl2, A[9] * inv - dl2 * dl2 + eps};
      if constexpr (GLOBAL) live = make_node(mu, cov, N / total, nd, nf);
      else live = make_nodef_fast(mu, cov, N / total, nf);
    }
    if (live) {
      if constexpr (GLOBAL) {
        NodeD& out = nodes[g];
        for (int i = 0; i < 3; ++i) out.mu[i] = nd.mu[i];
        for (int i = 0; i < 6; ++i) { out.cov[i] = nd.cov[i]; out.winv[i] = nd.winv[i]; }
        out.pi = nd.pi; out.c = nd.c; out.logdet = nd.logdet; out.live = 1;
        copy_nodef(tab[g], nf);
      }
      copy_nodef(ch[lane], nf);
    } else {
      if constexpr (GLOBAL) {
        nodes[g].live = 0; nodes[g].pi = 0.0;
        tab[g].flags = 0u;
      }
      ch[lane].flags = 0u;
    }
  }
  if constexpr (FRAME) {
    const uint64_t lm = __ballot(live);
    if (lm != 0ull) {
      const int r = __ffsll((long long)lm) - 1;
      const double f0 = __shfl(mu[0], r, 64), f1 = __shfl(mu[1], r, 64), f2 = __shfl(mu[2], r, 64);
      if (lane < 8) {
        float* q = fr->p[lane];
        q[0] = live ? (float)(mu[0] - f0) : 0.f;
        q[1] = live ? (float)(mu[1] - f1) : 0.f;
        q[2] = live ? (float)(mu[2] - f2) : 0.f;
        for (int i = 0; i < 6; ++i) q[3 + i] = live ? nf.w[i] : 0.f;
        q[9] = live ? nf.c : -INFINITY;
      }
      if (lane == 0) { fr->ref[0] = f0; fr->ref[1] = f1; fr->ref[2] = f2; }
    }
  }
}

__device__ __forceinline__ uint32_t live_mask(const NodeF* ch) {
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) m |= (ch[k].flags & F_LIVE) ? (1u << k) : 0u;
  return m;
}

static_assert(sizeof(EmFrame) <= kFrameBytes, "an E-step frame fits its record");

// The live children of a frame (a dead child has the constant -inf).
__device__ __forceinline__ uint32_t frame_live(const EmFrame& f) {
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) m |= (f.p[k][9] > -INFINITY) ? (1u << k) : 0u;
  return m;
}

// One EM iteration of the tiled (large) jobs: the E-step of the tile's points
// and the tile's partials of the 80 moment sums (FP64, value-major:
// part_next[v * pstride + tile]).  The children of the job (one set of 8 per
// tiled job, slot = Tile::pad, the job's place among the tiled jobs) come
// from one of two places:
//   INLINE: every block of the job folds the job's tile partials of the
//   previous iteration (part_prev) in the same fixed order and runs the same
//   FP64 M-step from ch_prev, so all its blocks hold bit-identical children,
//   and the job's first tile publishes them in ch_next (ping-pong buffers);
//   no launch between iterations, the fold repeated once per tile;
//   otherwise: the block reads the job's E-step frame (frames, kFrameBytes
//   per slot) that em_fold_kernel wrote after the previous iteration.
// The first iteration (first = 1) starts from the initial children in the
// scoring table, and the job's first tile publishes them in ch_next.
template <int NT, int KP, bool INLINE>
__global__ __launch_bounds__(NT) void em_tile_kernel(
    const float* __restrict__ xs, const float* __restrict__ ys, const float* __restrict__ zs,
    const Tile* __restrict__ tiles, const int* __restrict__ tile_ids, const Job* __restrict__ jobs,
    const NodeF* __restrict__ tab, const NodeF* __restrict__ ch_prev, NodeF* ch_next,
    const char* __restrict__ frames, const double* __restrict__ part_prev, double* part_next, size_t pstride,
    double eps, double min_mass, int first, const int* dn, int n) {
  constexpr int NR = NT / 16, NW = NT / 64;
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const int tix = tile_ids[w];
  const Tile tl = tiles[tix];
  const Job jb = jobs[tl.job];
  const int slot = tl.pad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ NodeF chs[8];
  __shared__ EmFrame fr;
  __shared__ float rows[NR][80];
  __shared__ double tot[INLINE ? 80 : 1];
  // this block's points are requested first; their latency overlaps the
  // fold or the frame
  PointCache<KP> pc;
  load_points<NT>(xs, ys, zs, tl.start, tl.end, tid, pc);
  if (first || INLINE) {
    if (tid < 8) copy_nodef(chs[tid], first ? tab[jb.child_base + tid] : ch_prev[(size_t)slot * 8 + tid]);
    if (INLINE && !first) {
      // wave w folds value groups w, w + NW, ... of 5 values each
      for (int v0 = 5 * wv; v0 < 80; v0 += 5 * NW) {
        double t[5];
        wave_fold<5, 4>(part_prev + (size_t)v0 * pstride + jb.tile_first, pstride, jb.ntiles, lane, t);
        if (lane == 0)
          for (int j = 0; j < 5; ++j) tot[v0 + j] = t[j];
      }
      __syncthreads();
      if (tid < 64) mstep_children<false, true>(tot, chs, nullptr, nullptr, 0, eps, min_mass, lane, &fr);
    }
    __syncthreads();
    if (tix == jb.tile_first && tid < 8) copy_nodef(ch_next[(size_t)slot * 8 + tid], chs[tid]);
    const uint32_t live0 = live_mask(chs);
    if (first) {
      if (live0) em_frame(chs, live0, fr, tid);
      else if (tid < 8) fr.p[tid][9] = -INFINITY;
    } else if (live0 == 0u && tid < 8) {
      fr.p[tid][9] = -INFINITY;  // the M-step left no live child
    }
  } else {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(frames + (size_t)slot * kFrameBytes);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&fr);
    for (int i = tid; i < (int)(sizeof(EmFrame) / 4); i += NT) dst[i] = src[i];
  }
  __syncthreads();
  const uint32_t live = frame_live(fr);
  float a[8][10];
  if (live) {
    em_range<NT, KP, false>(xs, ys, zs, tl.start, tl.end, tid, pc, fr, a);
  } else {
    for (int k = 0; k < 8; ++k)
      for (int v = 0; v < 10; ++v) a[k][v] = 0.f;
  }
  rows_store80(a, rows, tid);
  __syncthreads();
  for (int v = tid; v < 80; v += NT) {
    double t = 0.0;
    for (int q = 0; q < NR; ++q) t += (double)rows[q][v];
    part_next[(size_t)v * pstride + tix] = t;
  }
  __syncthreads();  // the block's LDS is reused by its next tile
  }
}

// The M-step of every tiled job between two iterations: one block of 4 waves
// per job (block b = the job's slot among the tiled jobs; small blocks find
// room beside the one-block-per-parent kernels that run at the same time);
// wave w folds the tile partials of values 20w .. 20w+19 in a fixed order,
// wave 0 runs the FP64 M-step of the children (ch, 8 per slot, updated in
// place) and the block writes the next iteration's E-step frame (frames,
// kFrameBytes per slot; every constant -inf when no child lives any more).
constexpr int kFoldThreads = 256;
__global__ __launch_bounds__(kFoldThreads) void em_fold_kernel(const int* __restrict__ job_ids,
                                                               const Job* __restrict__ jobs,
                                                               const double* __restrict__ partials, size_t pstride,
                                                               double eps, double min_mass, NodeF* ch, char* frames,
                                                               const int* dn, int n, const int* doff) {
  const int nw = work_count(dn, n), base = doff ? *doff : 0;
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Job jb = jobs[job_ids[base + w]];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ NodeF chs[8];
  __shared__ double tot[80];
  __shared__ EmFrame fr;
  if (tid < 8) copy_nodef(chs[tid], ch[(size_t)w * 8 + tid]);
  for (int v0 = 20 * wv; v0 < 20 * wv + 20; v0 += 5) {
    double t[5];
    wave_fold<5, 4>(partials + (size_t)v0 * pstride + jb.tile_first, pstride, jb.ntiles, lane, t);
    if (lane == 0)
      for (int j = 0; j < 5; ++j) tot[v0 + j] = t[j];
  }
  __syncthreads();
  if (tid < 64) mstep_children<false, true>(tot, chs, nullptr, nullptr, 0, eps, min_mass, lane, &fr);
  __syncthreads();
  if (tid < 8) {
    if (live_mask(chs) == 0u) {
      for (int i = 0; i < 9; ++i) fr.p[tid][i] = 0.f;
      fr.p[tid][9] = -INFINITY;
    }
    copy_nodef(ch[(size_t)w * 8 + tid], chs[tid]);
  }
  __syncthreads();
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&fr);
    uint32_t* dst = reinterpret_cast<uint32_t*>(frames + (size_t)w * kFrameBytes);
    for (int i = tid; i < (int)(sizeof(EmFrame) / 4); i += kFoldThreads) dst[i] = src[i];
  }
  __syncthreads();  // the block's LDS is reused by its next job
  }
}

constexpr int kMstepThreads = 1024;

// Final M-step of the tiled jobs after the last iteration: one block of 16
// waves per job (block b = the job's slot among the tiled jobs); wave w folds
// the tile partials of values 5w .. 5w+4 in a fixed order, then wave 0 runs
// the M-step from the children of that iteration (chsrc) and writes the node
// records.
__global__ __launch_bounds__(kMstepThreads) void em_mstep_kernel(const int* __restrict__ job_ids,
                                                                 const Job* __restrict__ jobs, NodeF* tab,
                                                                 NodeD* nodes, const double* __restrict__ partials,
                                                                 size_t pstride, double eps, double min_mass,
                                                                 const NodeF* __restrict__ chsrc, const int* dn, int n,
                                                                 const int* doff) {
  const int nw = work_count(dn, n), base = doff ? *doff : 0;
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Job jb = jobs[job_ids[base + w]];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ NodeF ch[8];
  __shared__ double tot[80];
  if (tid < 8) copy_nodef(ch[tid], chsrc[(size_t)w * 8 + tid]);
  double t[5];
  wave_fold<5, 8>(partials + (size_t)(5 * wv) * pstride + jb.tile_first, pstride, jb.ntiles, lane, t);
  if (lane == 0)
    for (int j = 0; j < 5; ++j) tot[5 * wv + j] = t[j];
  __syncthreads();
  if (tid < 64) mstep_children(tot, ch, tab, nodes, jb.child_base, eps, min_mass, lane);
  __syncthreads();
  }
}

// (Two waves per SIMD: with the children's parameters in scalar registers
// the compiler would otherwise trade occupancy 2 for 1 to keep more in flight,
// which is slower when many small parents share a compute unit.)
// All EM iterations of one job inside one block of NT threads: each thread
// accumulates the moments of every NT-th point of the job (the job's points
// stay in L1/L2 across iterations), the block reduces them (row butterflies,
// then the rows in FP64 in a fixed order) and wave 0 runs the FP64 M-step.
// One launch covers every iteration.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void em_block_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                      const float* __restrict__ zs, const int* __restrict__ job_ids,
                                                      const Job* __restrict__ jobs, NodeF* tab, NodeD* nodes,
                                                      int iters, double eps, double min_mass, const int* dn, int n,
                                                      const int* doff) {
  constexpr int NR = NT / 16;
  const int nw = work_count(dn, n), base = doff ? *doff : 0;
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Job jb = jobs[job_ids[base + w]];
  const int tid = threadIdx.x;
  __shared__ NodeF ch[8];
  __shared__ EmFrame fr;
  __shared__ float rows[NR][80];
  __shared__ double tot[80];
  if (tid < 8) copy_nodef(ch[tid], tab[jb.child_base + tid]);
  PointCache<8> pc;
  load_points<NT>(xs, ys, zs, jb.start, jb.start + jb.count, tid, pc);
  __syncthreads();
  {
    const uint32_t live0 = live_mask(ch);
    if (live0) em_frame(ch, live0, fr, tid);
  }
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    if (live_mask(ch) == 0u) break;
    float a[8][10];
    em_range<NT, 8, true>(xs, ys, zs, jb.start, jb.start + jb.count, tid, pc, fr, a);
    rows_store80(a, rows, tid);
    __syncthreads();
    for (int v = tid; v < 80; v += NT) {
      double t = 0.0;
      for (int q = 0; q < NR; ++q) t += (double)rows[q][v];
      tot[v] = t;
    }
    __syncthreads();
    if (tid < 64) {
      // intermediate iterations update the LDS children and the next frame;
      // the last one writes the node records
      if (it + 1 < iters) mstep_children<false, true>(tot, ch, nullptr, nullptr, 0, eps, min_mass, tid, &fr);
      else mstep_children<true, false>(tot, ch, tab, nodes, jb.child_base, eps, min_mass, tid);
    }
    __syncthreads();
  }
  // every child died in an intermediate iteration: record that
  if (live_mask(ch) == 0u && tid < 8) {
    const int g = jb.child_base + tid;
    nodes[g].live = 0; nodes[g].pi = 0.0;
    tab[g].flags = 0u;
  }
  __syncthreads();  // the block's LDS is reused by its next job
  }
}

// ---------------------------------------------------------------------------
// hard partition: most likely live child of every point, in FP64
// ---------------------------------------------------------------------------

// The FP64 scoring fields of a node read through the constant address space:
// the kernel never writes them, so reads at an address uniform over the block
// become scalar loads.
typedef const __attribute__((address_space(4))) NodeS ConstNodeS;

__device__ __forceinline__ double score64_c(const ConstNodeS* n, double p0, double p1, double p2) {
  const double d0 = p0 - n->mu[0], d1 = p1 - n->mu[1], d2 = p2 - n->mu[2];
  const double w0 = n->winv[0] * d0;
  const double w1 = n->winv[1] * d0 + n->winv[2] * d1;
  const double w2 = n->winv[3] * d0 + n->winv[4] * d1 + n->winv[5] * d2;
  return kLog2e * (n->c - 0.5 * (w0 * w0 + w1 * w1 + w2 * w2));
}

// Every point of a tile scores the 8 children of the tile's parent in FP64
// (full rate on CDNA4, as FP32 without packing) and takes the most likely
// live one (the lowest index on an exact tie; the first live child when no
// score is a number).  The children are the same for the whole block, so
// their records are read with scalar loads.
__global__ __launch_bounds__(64) void partition_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                       const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                       const Job* __restrict__ jobs, const NodeF* __restrict__ tab,
                                                       const NodeD* __restrict__ nodes, uint8_t* child_out,
                                                       int* tile_counts, const int* dn, int n) {
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Tile tl = tiles[w];
  const Job jb = jobs[tl.job];
  const int lane = threadIdx.x;
  uint32_t live = 0u;
#pragma unroll
  for (int k = 0; k < 8; ++k) live |= (tab[jb.child_base + k].flags & F_LIVE) ? (1u << k) : 0u;
  const ConstNodeS* S = (const ConstNodeS*)(nodes + jb.child_base);
  static_assert(sizeof(NodeD) % 8 == 0 && __builtin_offsetof(NodeD, c) == __builtin_offsetof(NodeS, c),
                "NodeS is the prefix of NodeD");
  int cnt[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int base = tl.start; base < tl.end; base += 64) {
    const int i = base + lane;
    const bool valid = i < tl.end;
    int bucket = 8;
    if (valid && live) {
      const double p0 = xs[i], p1 = ys[i], p2 = zs[i];
      double best = -INFINITY;
      int kb = -1;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (!(live & (1u << k))) continue;
        const double v = score64_c((const ConstNodeS*)((const __attribute__((address_space(4))) char*)S +
                                                       (size_t)k * sizeof(NodeD)),
                                   p0, p1, p2);
        if (kb < 0 || v > best) { best = v; kb = k; }
      }
      bucket = kb;
    }
    if (valid) child_out[i] = (uint8_t)bucket;
#pragma unroll
    for (int b = 0; b < 9; ++b) cnt[b] += __popcll(__ballot(valid && bucket == b));
  }
  if (lane < 9) {
    int v = cnt[0];
#pragma unroll
    for (int b = 1; b < 9; ++b) v = (lane == b) ? cnt[b] : v;
    tile_counts[(size_t)w * 9 + lane] = v;
  }
  }
}

// Per job: exclusive prefix of the bucket counts over its tiles, the start and
// size of every child's range, and the child partition sizes.
__global__ __launch_bounds__(64) void prefix_kernel(const Job* __restrict__ jobs, const int* __restrict__ tile_counts,
                                                    int* tile_base, NodeD* nodes, int2* lvl_info, const int* dn,
                                                    int n) {
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Job jb = jobs[w];
  const int lane = threadIdx.x;
  const int chunk = (jb.ntiles + 63) / 64;
  const int t0 = jb.tile_first + lane * chunk;
  const int t1 = min(jb.tile_first + jb.ntiles, t0 + chunk);
  int own[9], excl[9], tot[9];
#pragma unroll
  for (int b = 0; b < 9; ++b) own[b] = 0;
  for (int t = t0; t < t1; ++t)
#pragma unroll
    for (int b = 0; b < 9; ++b) own[b] += tile_counts[(size_t)t * 9 + b];
#pragma unroll
  for (int b = 0; b < 9; ++b) {
    int v = own[b];
    for (int d = 1; d < 64; d <<= 1) {
      int u = __shfl_up(v, d, 64);
      if (lane >= d) v += u;
    }
    excl[b] = v - own[b];
    tot[b] = __shfl(v, 63, 64);
  }
  int boff[9];
  boff[0] = 0;
#pragma unroll
  for (int b = 1; b < 9; ++b) boff[b] = boff[b - 1] + tot[b - 1];
  int run[9];
#pragma unroll
  for (int b = 0; b < 9; ++b) run[b] = jb.start + boff[b] + excl[b];
  for (int t = t0; t < t1; ++t)
#pragma unroll
    for (int b = 0; b < 9; ++b) {
      tile_base[(size_t)t * 9 + b] = run[b];
      run[b] += tile_counts[(size_t)t * 9 + b];
    }
  if (lane < 8) {
    int st = boff[0], ct = tot[0];
#pragma unroll
    for (int b = 1; b < 8; ++b) {
      st = (lane == b) ? boff[b] : st;
      ct = (lane == b) ? tot[b] : ct;
    }
    nodes[jb.child_base + lane].count = ct;
    lvl_info[jb.child_lvl + lane] = make_int2(jb.start + st, ct);
  }
  }
}

// Stable 9-way split of each job's range by child (8 = no live child): moves
// the points, the original indices and writes the level's labels.
__global__ __launch_bounds__(64) void scatter_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                     const float* __restrict__ zs, const int* __restrict__ perm,
                                                     const Tile* __restrict__ tiles, const Job* __restrict__ jobs,
                                                     const TreeDev* __restrict__ trees, const uint8_t* __restrict__ child,
                                                     const int* __restrict__ tile_base, float* xo, float* yo, float* zo,
                                                     int* perm_out, int32_t* labels, int level, int64_t level_off,
                                                     const int* dn, int n) {
  const int nw = work_count(dn, n);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
  const Tile tl = tiles[w];
  const Job jb = jobs[tl.job];
  const TreeDev& T = trees[jb.tree];
  const int lane = threadIdx.x;
  __shared__ int base[9];
  if (lane < 9) base[lane] = tile_base[(size_t)w * 9 + lane];
  __syncthreads();
  const int local_child0 = (int)(jb.child_base - T.node_base - level_off);
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int b0 = tl.start; b0 < tl.end; b0 += 64) {
    const int i = b0 + lane;
    const bool valid = i < tl.end;
    const int b = valid ? (int)child[i] : 15;
    int rank = 0, dst = 0;
    int add[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      unsigned long long msk = __ballot(b == v);
      if (b == v) rank = __popcll(msk & lt);
      add[v] = __popcll(msk);
    }
    if (valid) dst = base[b] + rank;
    __syncthreads();
    if (lane < 9) {
      int v = add[0];
#pragma unroll
      for (int u = 1; u < 9; ++u) v = (lane == u) ? add[u] : v;
      base[lane] += v;
    }
    if (valid) {
      const int src = perm ? perm[i] : i;
      xo[dst] = xs[i]; yo[dst] = ys[i]; zo[dst] = zs[i];
      perm_out[dst] = src;
      if (b < 8) labels[T.label_base + (int64_t)level * T.n_points + (src - T.point_off)] = local_child0 + b;
    }
    __syncthreads();
  }
  __syncthreads();
  }
}

// Eigen-decomposition, complexity and global weight of the new level's nodes;
// the parent learns whether it has live children.
__global__ __launch_bounds__(64) void finalize_level_kernel(const Job* __restrict__ jobs, int njobs, NodeD* nodes,
                                                            NodeF* tab, const int* dn) {
  const int nj = work_count(dn, njobs);
  // the loop bound is uniform over the wave, so the ballot below sees all lanes
  for (int base = blockIdx.x * 64; base < 8 * nj; base += gridDim.x * 64) {
  const int gid = base + threadIdx.x;
  const int j = gid >> 3, k = gid & 7;
  const bool valid = j < nj;
  bool live = false;
  Job jb;
  if (valid) {
    jb = jobs[j];
    live = nodes[jb.child_base + k].live != 0;
  }
  const unsigned long long bal = __ballot(live);
  if (!valid) continue;
  const int lane = threadIdx.x;
  const bool any = ((bal >> (lane & ~7)) & 0xFFull) != 0ull;
  if (k == 0 && jb.parent >= 0) {
    nodes[jb.parent].has_children = any ? 1 : 0;
    if (any) tab[jb.parent].flags |= F_HASCH;
  }
  NodeD& nd = nodes[jb.child_base + k];
  nd.has_children = 0;
  if (!live) {
    nd.count = 0;
    continue;
  }
  double lam[3], ev[9];
  eig_sym3(nd.cov, lam, ev);
  for (int i = 0; i < 3; ++i) nd.lam[i] = lam[i];
  for (int i = 0; i < 9; ++i) nd.evec[i] = ev[i];
  nd.kappa = lam[2] / (lam[0] + lam[1] + lam[2]);
  nd.pig = nd.pi * (jb.parent >= 0 ? nodes[jb.parent].pig : 1.0);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// level planning on the device (for construction captured in one graph)
// ---------------------------------------------------------------------------

// Job of parent item i of a level: item i is entry i / per of the level's tree
// list, parent k = i % per of that tree (at level 0 the tree root itself).
__device__ __forceinline__ void plan_item(int64_t i, int per, int level, int64_t loff_prev, int64_t loff_cur,
                                          const LevelTree* __restrict__ lt, const int2* __restrict__ lvl_prev,
                                          const TreeDev* __restrict__ trees, Job& j) {
  const int e = (int)(i / per), k = (int)(i % per);
  const LevelTree L = lt[e];
  const TreeDev& T = trees[L.b];
  j.tree = L.b;
  if (level == 0) {
    j.start = (int32_t)T.point_off;
    j.count = T.n_points;
    j.parent = -1;
    j.child_base = (int32_t)T.node_base;
    j.child_lvl = L.cur_base;
  } else {
    const int2 inf = lvl_prev[L.prev_base + k];
    j.start = inf.x;
    j.count = inf.y;
    j.parent = (int32_t)(T.node_base + loff_prev + k);
    j.child_base = (int32_t)(T.node_base + loff_cur + 8 * (int64_t)k);
    j.child_lvl = L.cur_base + 8 * k;
  }
}

// The plan of one level, as the host planner makes it and in the same order:
// a job per parent with points (every tree root at level 0), in tree order
// then parent order; the job ids class by class (class by point count:
// thresholds b64 / b256 / b512, else tiled); tiles of tpts points, job after
// job; the tile ids of the tiled jobs; the slot of a tiled job (its rank among
// the tiled jobs) in its tiles' pad.  One block; two passes over the parents
// (totals, then an ordered block scan).  Sets plan[PL_ERR] instead of writing
// past max_jobs / max_tiles.
constexpr int kPlanThreads = 1024;
__global__ __launch_bounds__(kPlanThreads) void plan_level_kernel(
    const LevelTree* __restrict__ lt, int nlt, int per, int level, int64_t loff_prev, int64_t loff_cur,
    const int2* __restrict__ lvl_prev, const TreeDev* __restrict__ trees, int b64, int b256, int b512,
    int target_tiles, int min_tile, int max_tile, int max_jobs, int max_tiles, Job* jobs, int* job_ids, Tile* tiles,
    int* tile_ids, int* plan) {
  constexpr int NV = 7, NW = kPlanThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t total = (int64_t)nlt * per;
  __shared__ unsigned long long s_points;
  __shared__ int s_cls[4], s_off[5], s_tpts, s_err;
  __shared__ int s_woff[NW][NV], s_btot[NV], s_carry[NV];
  // items of the current chunk, for writing its tiles with the whole block:
  // chunk-local first tile, global first tile, first tile id (tiled jobs),
  // job, start, points, slot (tiled) or -1
  __shared__ int s_tl[kPlanThreads], s_tg[kPlanThreads], s_bf[kPlanThreads], s_jid[kPlanThreads],
      s_st[kPlanThreads], s_ct[kPlanThreads], s_sl[kPlanThreads];
  if (tid == 0) {
    s_points = 0ull;
    s_err = 0;
    for (int c = 0; c < 4; ++c) s_cls[c] = 0;
    for (int k = 0; k < NV; ++k) s_carry[k] = 0;
  }
  __syncthreads();
  auto cls_of = [&](int count) { return count <= b64 ? 0 : count <= b256 ? 1 : count <= b512 ? 2 : 3; };
  // pass 1: points of the level and jobs per class
  {
    unsigned long long pts = 0ull;
    int cl[4] = {0, 0, 0, 0};
    for (int64_t i = tid; i < total; i += kPlanThreads) {
      Job j;
      plan_item(i, per, level, loff_prev, loff_cur, lt, lvl_prev, trees, j);
      if (level == 0 || j.count > 0) {
        pts += (unsigned long long)j.count;
        cl[cls_of(j.count)] += 1;
      }
    }
    atomicAdd(&s_points, pts);
    for (int c = 0; c < 4; ++c) atomicAdd(&s_cls[c], cl[c]);
  }
  __syncthreads();
  if (tid == 0) {
    int64_t t = (int64_t)s_points / (target_tiles > 1 ? target_tiles : 1);
    t = (t + 63) / 64 * 64;
    t = t > min_tile ? t : min_tile;
    t = t < max_tile ? t : max_tile;
    s_tpts = (int)t;
    s_off[0] = 0;
    for (int c = 0; c < 4; ++c) s_off[c + 1] = s_off[c] + s_cls[c];
  }
  __syncthreads();
  const int tpts = s_tpts;
  // pass 2: ordered exclusive scan of (job, job of class 0..3, tiles, tiles of
  // tiled jobs) over the parents, 1024 at a time
  for (int64_t base = 0; base < total; base += kPlanThreads) {
    const int64_t i = base + tid;
    Job j;
    j.count = 0;
    bool valid = false;
    if (i < total) {
      plan_item(i, per, level, loff_prev, loff_cur, lt, lvl_prev, trees, j);
      valid = (level == 0 || j.count > 0);
    }
    const int c = valid ? cls_of(j.count) : -1;
    const int ntl = valid ? (j.count + tpts - 1) / tpts : 0;
    int v[NV] = {valid ? 1 : 0, c == 0, c == 1, c == 2, c == 3, ntl, c == 3 ? ntl : 0};
    int inc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      int x = v[k];
      for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(x, d, 64);
        if (lane >= d) x += u;
      }
      inc[k] = x;
      if (lane == 63) s_woff[wv][k] = x;
    }
    __syncthreads();
    if (tid < NV) {
      int run = 0;
      for (int w = 0; w < NW; ++w) {
        const int x = s_woff[w][tid];
        s_woff[w][tid] = run;
        run += x;
      }
      s_btot[tid] = run;
    }
    __syncthreads();
    {
      int ex[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) ex[k] = s_carry[k] + s_woff[wv][k] + inc[k] - v[k];
      const int jid = ex[0], pos = valid ? ex[1 + c] : 0, tfirst = ex[5], bfirst = ex[6];
      s_tl[tid] = tfirst - s_carry[5];
      s_jid[tid] = -1;
      if (valid) {
        if (jid >= max_jobs || s_off[c] + pos >= max_jobs || tfirst + ntl > max_tiles) {
          s_err = 1;
        } else {
          j.tile_first = tfirst;
          j.ntiles = ntl;
          jobs[jid] = j;
          job_ids[s_off[c] + pos] = jid;
          s_tg[tid] = tfirst;
          s_bf[tid] = bfirst;
          s_jid[tid] = jid;
          s_st[tid] = j.start;
          s_ct[tid] = j.count;
          s_sl[tid] = (c == 3) ? pos : -1;
        }
      }
    }
    __syncthreads();
    // the chunk's tiles, one per thread: tile u belongs to the last item whose
    // chunk-local first tile is <= u (items without tiles share the offset of
    // the next one)
    const int nct = s_btot[5];
    for (int u = tid; u < nct; u += kPlanThreads) {
      int lo = 0, hi = kPlanThreads - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_tl[mid] <= u) lo = mid;
        else hi = mid - 1;
      }
      if (s_jid[lo] < 0) continue;  // an overflowed item (s_err is set)
      const int t = u - s_tl[lo];
      Tile T;
      T.start = s_st[lo] + t * tpts;
      T.end = min(s_st[lo] + s_ct[lo], T.start + tpts);
      T.job = s_jid[lo];
      T.pad = s_sl[lo] >= 0 ? s_sl[lo] : 0;
      tiles[s_tg[lo] + t] = T;
      if (s_sl[lo] >= 0) tile_ids[s_bf[lo] + t] = s_tg[lo] + t;
    }
    __syncthreads();
    if (tid < NV) s_carry[tid] += s_btot[tid];
    __syncthreads();
  }
  if (tid == 0) {
    // after an overflow the level does no work (every count 0); the host
    // reports plan[PL_ERR]
    const int ok = s_err ? 0 : 1;
    plan[PL_NJOBS] = ok * s_carry[0];
    plan[PL_NTILES] = ok * s_carry[5];
    plan[PL_NBIG] = ok * s_carry[6];
    for (int c = 0; c < 4; ++c) plan[PL_CLS_N + c] = ok * s_cls[c];
    for (int c = 0; c < 5; ++c) plan[PL_CLS_OFF + c] = ok * s_off[c];
    plan[PL_TPTS] = tpts;
    plan[PL_ERR] = s_err;
  }
}

void launch_plan_level(const LevelTree* lt, int nlt, int per, int level, int64_t loff_prev, int64_t loff_cur,
                       const int2* lvl_prev, const TreeDev* trees, int b64, int b256, int b512, int target_tiles,
                       int min_tile, int max_tile, int max_jobs, int max_tiles, Job* jobs, int* job_ids, Tile* tiles,
                       int* tile_ids, int* plan, hipStream_t s) {
  hipLaunchKernelGGL(plan_level_kernel, dim3(1), dim3(kPlanThreads), 0, s, lt, nlt, per, level, loff_prev, loff_cur,
                     lvl_prev, trees, b64, b256, b512, target_tiles, min_tile, max_tile, max_jobs, max_tiles, jobs,
                     job_ids, tiles, tile_ids, plan);
}

// Launchers.  With a device count dn (a level planned on the device) the
// kernels read their number of work items from *dn and the n given here is
// the (fixed) grid; without it n is the number of work items, one block each.
void launch_root(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles, const Job* jobs,
                 int njobs, TreeDev* trees, double* partials, size_t pstride, double eps, hipStream_t s,
                 const int* dntiles, const int* dnjobs) {
  hipLaunchKernelGGL(root_mean_kernel, dim3(ntiles), dim3(64), 0, s, xs, ys, zs, tiles, partials, pstride, dntiles,
                     ntiles);
  hipLaunchKernelGGL(root_mean_fold_kernel, dim3(njobs), dim3(64), 0, s, jobs, trees, partials, pstride, dnjobs,
                     njobs);
  hipLaunchKernelGGL(root_cov_kernel, dim3(ntiles), dim3(64), 0, s, xs, ys, zs, tiles, jobs, trees, partials, pstride,
                     dntiles, ntiles);
  hipLaunchKernelGGL(root_cov_fold_kernel, dim3(njobs), dim3(64), 0, s, jobs, trees, partials, pstride, eps, dnjobs,
                     njobs);
}

void launch_init_children(const Job* jobs, int njobs, const TreeDev* trees, NodeD* nodes, NodeF* tab, double eps,
                          hipStream_t s, const int* dn) {
  int threads = njobs * 8;
  hipLaunchKernelGGL(init_children_kernel, dim3((threads + 63) / 64), dim3(64), 0, s, jobs, njobs, trees, nodes, tab,
                     eps, dn);
}

void launch_em_tile(int nt, const float* xs, const float* ys, const float* zs, const Tile* tiles, const int* tile_ids,
                    int n, const Job* jobs, const NodeF* tab, const NodeF* ch_prev, NodeF* ch_next, const void* frames,
                    const double* part_prev, double* part_next, size_t pstride, double eps, double min_mass,
                    int first, bool inline_fold, hipStream_t s, const int* dn) {
  const char* fr = static_cast<const char*>(frames);
#define HGMM_EM_TILE(NT_, KP_, IN_)                                                                               \
  hipLaunchKernelGGL((em_tile_kernel<NT_, KP_, IN_>), dim3(n), dim3(NT_), 0, s, xs, ys, zs, tiles, tile_ids, jobs, \
                     tab, ch_prev, ch_next, fr, part_prev, part_next, pstride, eps, min_mass, first, dn, n)
  if (nt == 1024) {
    if (inline_fold) HGMM_EM_TILE(1024, 2, true); else HGMM_EM_TILE(1024, 2, false);
  } else if (nt == 512) {
    if (inline_fold) HGMM_EM_TILE(512, 4, true); else HGMM_EM_TILE(512, 4, false);
  } else {
    if (inline_fold) HGMM_EM_TILE(256, 4, true); else HGMM_EM_TILE(256, 4, false);
  }
#undef HGMM_EM_TILE
}

void launch_em_fold(const int* job_ids, int n, const Job* jobs, const double* partials, size_t pstride, double eps,
                    double min_mass, NodeF* ch, void* frames, hipStream_t s, const int* dn, const int* doff) {
  hipLaunchKernelGGL(em_fold_kernel, dim3(n), dim3(kFoldThreads), 0, s, job_ids, jobs, partials, pstride, eps,
                     min_mass, ch, static_cast<char*>(frames), dn, n, doff);
}

void launch_em_mstep(const int* job_ids, int n, const Job* jobs, NodeF* tab, NodeD* nodes, const double* partials,
                     size_t pstride, double eps, double min_mass, const NodeF* chsrc, hipStream_t s, const int* dn,
                     const int* doff) {
  hipLaunchKernelGGL(em_mstep_kernel, dim3(n), dim3(kMstepThreads), 0, s, job_ids, jobs, tab, nodes, partials,
                     pstride, eps, min_mass, chsrc, dn, n, doff);
}

void launch_em_block(int nt, const float* xs, const float* ys, const float* zs, const int* job_ids, int n,
                     const Job* jobs, NodeF* tab, NodeD* nodes, int iters, double eps, double min_mass,
                     hipStream_t s, const int* dn, const int* doff) {
  if (n <= 0) return;
  if (nt == 64)
    hipLaunchKernelGGL(em_block_kernel<64>, dim3(n), dim3(64), 0, s, xs, ys, zs, job_ids, jobs, tab, nodes, iters,
                       eps, min_mass, dn, n, doff);
  else if (nt == 256)
    hipLaunchKernelGGL(em_block_kernel<256>, dim3(n), dim3(256), 0, s, xs, ys, zs, job_ids, jobs, tab, nodes, iters,
                       eps, min_mass, dn, n, doff);
  else
    hipLaunchKernelGGL(em_block_kernel<512>, dim3(n), dim3(512), 0, s, xs, ys, zs, job_ids, jobs, tab, nodes, iters,
                       eps, min_mass, dn, n, doff);
}

void launch_partition(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                      const Job* jobs, const NodeF* tab, const NodeD* nodes, uint8_t* child, int* tile_counts,
                      hipStream_t s, const int* dn) {
  hipLaunchKernelGGL(partition_kernel, dim3(ntiles), dim3(64), 0, s, xs, ys, zs, tiles, jobs, tab, nodes, child,
                     tile_counts, dn, ntiles);
}

void launch_prefix(const Job* jobs, int njobs, const int* tile_counts, int* tile_base, NodeD* nodes, int2* lvl_info,
                   hipStream_t s, const int* dn) {
  hipLaunchKernelGGL(prefix_kernel, dim3(njobs), dim3(64), 0, s, jobs, tile_counts, tile_base, nodes, lvl_info, dn,
                     njobs);
}

void launch_scatter(const float* xs, const float* ys, const float* zs, const int* perm, const Tile* tiles, int ntiles,
                    const Job* jobs, const TreeDev* trees, const uint8_t* child, const int* tile_base, float* xo,
                    float* yo, float* zo, int* perm_out, int32_t* labels, int level, int64_t level_off,
                    hipStream_t s, const int* dn) {
  hipLaunchKernelGGL(scatter_kernel, dim3(ntiles), dim3(64), 0, s, xs, ys, zs, perm, tiles, jobs, trees, child,
                     tile_base, xo, yo, zo, perm_out, labels, level, level_off, dn, ntiles);
}

void launch_finalize_level(const Job* jobs, int njobs, NodeD* nodes, NodeF* tab, hipStream_t s, const int* dn) {
  int threads = njobs * 8;
  hipLaunchKernelGGL(finalize_level_kernel, dim3((threads + 63) / 64), dim3(64), 0, s, jobs, njobs, nodes, tab, dn);
}

}  // namespace hgmm
