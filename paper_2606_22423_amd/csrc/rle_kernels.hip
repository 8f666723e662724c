// Fused scan of a run-length encoded column.  Runs never cross a 1024-value
// block, so a wavefront takes blocks k = w, w + W, ... (W wavefronts, a
// wave-uniform index), tests the block's zone map (skip; with the all-match
// shortcut a block inside the predicate contributes its value count and the
// sum of value x length of its runs without testing them), and otherwise its
// lanes take the block's runs 64 at a time: one compare per run, COUNT += len,
// SUM += value * len (mod 2^64).  Per-lane partials meet in one wave reduction
// and three 64-bit atomics per wavefront.
#include "device_common.h"
#include "rle_kernels.h"

namespace scan_dev {

__global__ __launch_bounds__(256) void rle_scan_kernel(const RleParams p) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t tw = (uint64_t)gridDim.x * (blockDim.x >> 6);
  uint64_t count = 0, sum = 0, blocks = 0;
  for (uint64_t k = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave; k < p.nb; k += tw) {
    bool inside = false;
    if (p.use_zm) {
      const int64_t mn = p.zmin[k], mx = p.zmax[k];
      if (mx < p.lo || mn >= p.hi) continue;
      inside = p.use_am && mn >= p.lo && mx < p.hi;
    }
    blocks += inside ? 0u : 1u;
    const uint64_t r0 = p.block_run[k], r1 = p.block_run[k + 1];
    for (uint64_t r = r0 + lane; r < r1; r += 64u) {
      const uint32_t v = p.run_value[r];
      const uint32_t len = p.run_len[r];
      const bool ok = inside || ((int64_t)v >= p.lo && (int64_t)v < p.hi);
      count += ok ? len : 0u;
      sum += ok ? (uint64_t)v * len : 0ull;
    }
  }
  count = wave_sum_u64(count);
  sum = wave_sum_u64(sum);
  if (lane == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&p.out->count), (unsigned long long)count);
    atomicAdd(reinterpret_cast<unsigned long long*>(&p.out->sum), (unsigned long long)sum);
    atomicAdd(reinterpret_cast<unsigned long long*>(&p.out->blocks_read), (unsigned long long)blocks);
  }
}

__global__ void rle_clear_kernel(Result* out) {
  if (threadIdx.x == 0) *out = Result{0, 0, 0, 0, 0, 0};
}

hipError_t launch_rle_scan(const RleParams& p, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(rle_clear_kernel, dim3(1), dim3(64), 0, st, p.out);
  hipLaunchKernelGGL(rle_scan_kernel, dim3(grid), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace scan_dev
