// Fold of the per-work-group partials into a scan's result (see write_partial
// in device_common.h): one work-group, launched after the scan on its stream.
#include "device_common.h"

namespace scan_dev {

// Each thread keeps eight partials' loads in flight (two 16-byte loads per
// partial) before it adds them (one round trip for up to 2048 partials).
__global__ __launch_bounds__(256) void fold_partials_kernel(const Partial* __restrict__ partials, uint32_t n,
                                                            Result* out, uint64_t blocks_total, int32_t strategy) {
  __shared__ uint64_t red[4][3];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  constexpr uint32_t kPer = 8;
  const uint4* q4 = reinterpret_cast<const uint4*>(partials);
  uint64_t c = 0, t = 0, b = 0;
  for (uint32_t i0 = 0; i0 < n; i0 += blockDim.x * kPer) {
    uint4 x[kPer], y[kPer];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint32_t i = i0 + threadIdx.x + j * blockDim.x;
      x[j] = i < n ? q4[2u * i] : make_uint4(0u, 0u, 0u, 0u);       // count, sum
      y[j] = i < n ? q4[2u * i + 1u] : make_uint4(0u, 0u, 0u, 0u);  // blocks, pad
    }
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      c += ((uint64_t)x[j].y << 32) | x[j].x;
      t += ((uint64_t)x[j].w << 32) | x[j].z;
      b += ((uint64_t)y[j].y << 32) | y[j].x;
    }
  }
  c = wave_sum_u64(c);
  t = wave_sum_u64(t);
  b = wave_sum_u64(b);
  if (lane == 0) {
    red[wave][0] = c;
    red[wave][1] = t;
    red[wave][2] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < 4u; ++w) {
      red[0][0] += red[w][0];
      red[0][1] += red[w][1];
      red[0][2] += red[w][2];
    }
    Result r;
    r.count = red[0][0];
    r.sum = (int64_t)red[0][1];
    r.blocks_read = red[0][2];
    r.blocks_total = blocks_total;
    r.strategy_used = strategy;
    r.status = 0;
    *out = r;
  }
}

hipError_t launch_fold(const Partial* partials, uint32_t n, Result* out, uint64_t blocks_total, int32_t strategy,
                       hipStream_t st) {
  hipLaunchKernelGGL(fold_partials_kernel, dim3(1), dim3(256), 0, st, partials, n, out, blocks_total, strategy);
  return hipGetLastError();
}

// A result known on the host (an empty scan) written to device memory by a
// kernel, so that no host buffer has to outlive the call.
__global__ void write_result_kernel(Result* out, Result r) {
  if (threadIdx.x == 0) *out = r;
}

hipError_t launch_write_result(Result* out, const Result& r, hipStream_t st) {
  hipLaunchKernelGGL(write_result_kernel, dim3(1), dim3(64), 0, st, out, r);
  return hipGetLastError();
}

}  // namespace scan_dev
