// Fused scan of a run-length encoded column.  Runs never cross a 1024-value
// block, and a block's zone map only ever agrees with a test of its runs: a
// skipped block (max < lo or min >= hi) has no run that passes, a block
// inside the predicate (the all-match case) has no run that fails.  So the
// zone maps decide which runs are read and how blocks_read is counted, never
// the result.
//
// Without zone maps the runs stream through the lanes in one flat,
// grid-strided pass.  With them, a wavefront takes chunks of 64 consecutive
// blocks: lane j classifies block
// k0 + j from its zone map (one coalesced load per chunk), the chunk's
// blocks_read is a popcount of the ballot of tested blocks, and the runs of
// the span from the first to the last block not skipped stream through the
// lanes, four consecutive runs per lane and load (one compare per run, COUNT += len,
// SUM += value * len mod 2^64).  Per-lane partials meet in a work-group
// reduction, one partial per work-group, folded by a one-work-group kernel
// launched after it (no same-address atomics).
#include "device_common.h"
#include "rle_kernels.h"

namespace scan_dev {

namespace {

constexpr uint32_t kRleUnroll = 4;  // groups of four runs per lane in flight

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

// Runs q .. q + 3 (q a multiple of 4): those in [r0, r1) are tested.  One
// 16-byte value load and one 8-byte length load when all four runs exist
// (q + 4 <= total), single loads otherwise.
__device__ __forceinline__ void take_runs(const RleParams& p, uint64_t q, uint64_t r0, uint64_t r1, uint64_t total,
                                          uint64_t& count, uint64_t& sum) {
  if (q >= r1) return;
  uint32_t v[4], l[4];
  if (q + 4u <= total) {
    // adjacent lanes read adjacent runs: whole lines, streamed (non-temporal)
    const u32x4 vv = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p.run_value + q));
    const u16x4 ll = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(p.run_len + q));
    v[0] = vv.x, v[1] = vv.y, v[2] = vv.z, v[3] = vv.w;
    l[0] = ll.x, l[1] = ll.y, l[2] = ll.z, l[3] = ll.w;
  } else {
#pragma unroll
    for (uint32_t j = 0; j < 4u; ++j) {
      v[j] = q + j < total ? p.run_value[q + j] : 0u;
      l[j] = q + j < total ? p.run_len[q + j] : 0u;
    }
  }
#pragma unroll
  for (uint32_t j = 0; j < 4u; ++j) {
    const uint64_t r = q + j;
    const bool ok = r >= r0 && r < r1 && (int64_t)v[j] >= p.lo && (int64_t)v[j] < p.hi;
    count += ok ? l[j] : 0u;
    sum += ok ? (uint64_t)v[j] * l[j] : 0ull;
  }
}

}  // namespace

__global__ __launch_bounds__(512) void rle_scan_kernel(const RleParams p) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t tw = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const uint64_t nchunks = (p.nb + 63) / 64;
  const uint64_t total = p.block_run[p.nb];  // runs in the column
  uint64_t count = 0, sum = 0, blocks = 0;
  if (!p.use_zm) {
    // no zone maps: one flat pass over all runs, every block tested
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    blocks = gw == 0 ? p.nb : 0u;
    for (uint64_t q = gw * 256ull * kRleUnroll + 4ull * lane; q < total; q += tw * 256ull * kRleUnroll) {
#pragma unroll
      for (uint32_t u = 0; u < kRleUnroll; ++u) take_runs(p, q + 256ull * u, 0, total, total, count, sum);
    }
    write_partial(p.partials, wave_sum_u64(count), sum, blocks);
    return;
  }
  for (uint64_t c = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave; c < nchunks; c += tw) {
    const uint64_t k0 = c * 64u;
    const uint64_t k = k0 + lane;
    const bool in = k < p.nb;
    // 0: skipped, 1: tested run by run, 2: inside the predicate (all-match)
    uint32_t cls = in ? 1u : 0u;
    if (in && p.use_zm) {
      const int64_t mn = p.zmin[k], mx = p.zmax[k];
      if (mx < p.lo || mn >= p.hi) cls = 0u;
      else if (p.use_am && mn >= p.lo && mx < p.hi) cls = 2u;
    }
    // ballots in uniform control flow: every lane takes part, and `blocks`
    // stays the same in every lane
    const uint64_t tested = ballot(cls == 1u);
    const uint64_t live = ballot(cls != 0u);
    blocks += (uint64_t)__builtin_popcountll(tested);
    if (live == 0) continue;
    const uint32_t first = (uint32_t)__builtin_ctzll(live);
    const uint32_t last = 63u - (uint32_t)__builtin_clzll(live);
    // runs of blocks first .. last (skipped blocks in between add nothing),
    // lane l taking runs q .. q + 3 from the 4-aligned start on
    const uint64_t r0 = p.block_run[k0 + first];
    const uint64_t r1 = p.block_run[k0 + last + 1u];
    for (uint64_t q = (r0 & ~3ull) + 4ull * lane; q < r1; q += 256ull * kRleUnroll) {
#pragma unroll
      for (uint32_t u = 0; u < kRleUnroll; ++u) take_runs(p, q + 256ull * u, r0, r1, total, count, sum);
    }
  }
  write_partial(p.partials, wave_sum_u64(count), sum, blocks);
}

__global__ void rle_clear_kernel(Result* out, uint64_t blocks_total, int32_t strategy_used) {
  if (threadIdx.x == 0) *out = Result{0, 0, 0, blocks_total, strategy_used, 0};
}

hipError_t launch_rle_scan(const RleParams& p, uint32_t grid, hipStream_t st) {
  if (p.empty) {
    hipLaunchKernelGGL(rle_clear_kernel, dim3(1), dim3(64), 0, st, p.out, p.nb, p.strategy_used);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(rle_scan_kernel, dim3(grid), dim3(512), 0, st, p);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? launch_fold(p.partials, grid, p.out, p.nb, p.strategy_used, st) : e;
}

}  // namespace scan_dev
