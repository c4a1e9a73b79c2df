// Spatial ordering of the moving clouds for registration.  Points of each pair
// are sorted by the 30-bit Morton code of their position in the model tree's
// frame (origin, extent), with the pair index in the key's upper 32 bits so
// that every pair keeps its own contiguous range.  Neighbouring lanes of a
// wavefront then tend to stop at the same tree node, so the descent's
// per-node aggregation inside a wave merges more points per flush.  Rigid
// motion keeps the ordering coherent at every iteration; the sort runs once
// per registration call.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "hgmm_dev.h"
#include "hgmm_host.h"

namespace hgmm {

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t quant10(double x, double o, double inv_ext) {
  double u = (x - o) * inv_ext + 0.5;
  u = fmin(fmax(u, 0.0), 0.999999);
  return (uint32_t)(u * 1024.0);
}

__global__ __launch_bounds__(256) void morton_keys_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                                          const float* __restrict__ zs, const Tile* __restrict__ tiles,
                                                          const TreeDev* __restrict__ trees, uint64_t* keys,
                                                          int* vals) {
  const Tile tl = tiles[blockIdx.x];
  const TreeDev& T = trees[tl.job];
  const double inv = T.extent > 0.0 ? 1.0 / T.extent : 1.0;
  for (int i = tl.start + (int)threadIdx.x; i < tl.end; i += blockDim.x) {
    const uint32_t m = spread10(quant10(xs[i], T.origin[0], inv)) | (spread10(quant10(ys[i], T.origin[1], inv)) << 1) |
                       (spread10(quant10(zs[i], T.origin[2], inv)) << 2);
    keys[i] = ((uint64_t)(uint32_t)tl.job << 32) | m;
    vals[i] = i;
  }
}

__global__ void gather_points_kernel(const float* __restrict__ xs, const float* __restrict__ ys,
                                     const float* __restrict__ zs, const int* __restrict__ perm, int64_t n, float* xo,
                                     float* yo, float* zo) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = perm[j];
  xo[j] = xs[i];
  yo[j] = ys[i];
  zo[j] = zs[i];
}

static int key_bits(int npairs) {
  int b = 0;
  while ((1ll << b) < (long long)npairs) ++b;
  return 30 + (b > 0 ? 2 + b : 2);  // bits 30-31 are zero; the pair index starts at bit 32
}

size_t sort_temp_bytes(int64_t n, int npairs) {
  size_t bytes = 0;
  if (n <= 0) return 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, (int)n, 0, key_bits(npairs));
  return bytes;
}

hipError_t launch_sort_points(const float* xs, const float* ys, const float* zs, const Tile* tiles, int ntiles,
                              const TreeDev* trees, int npairs, int64_t n, uint64_t* keys, uint64_t* keys_out,
                              int* vals, int* perm, void* temp, size_t temp_bytes, float* xo, float* yo, float* zo,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(morton_keys_kernel, dim3(ntiles), dim3(256), 0, s, xs, ys, zs, tiles, trees, keys, vals);
  size_t bytes = temp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, bytes, (const uint64_t*)keys, keys_out, (const int*)vals,
                                                    perm, (int)n, 0, key_bits(npairs), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gather_points_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xs, ys, zs, perm, n, xo,
                     yo, zo);
  return hipGetLastError();
}

}  // namespace hgmm
