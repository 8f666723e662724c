// Bandwidth probes: the sequential-read maximum (the beta the scan's HBM
// fraction is measured against), STREAM triad, and a cache-flush writer.
// The paper measures beta per machine both as STREAM-Triad and as an
// empirical sequential-read maximum over buffers much larger than the last
// cache level, and reports f against the read maximum.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scan_dev {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Grid-stride read of n16 16-byte words, U loads in flight per thread.  The
// conditional store on a data-dependent value keeps the loads alive.
template <int U>
__global__ __launch_bounds__(1024) void beta_read_kernel(const uint4* __restrict__ buf, uint64_t n16,
                                                          uint64_t* sink) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    u32x4 v[U];
    const u32x4* src = reinterpret_cast<const u32x4*>(buf);
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n16; i += stride) {
    const uint4 v = buf[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

__global__ __launch_bounds__(256) void beta_triad_kernel(float4* __restrict__ a, const float4* __restrict__ b,
                                                          const float4* __restrict__ c, float s, uint64_t n4) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 x = b[i], y = c[i];
    a[i] = make_float4(x.x + s * y.x, x.y + s * y.y, x.z + s * y.z, x.w + s * y.w);
  }
}

// Reads the scratch buffer so that its lines displace whatever the caches
// held.  Reading rather than writing leaves the caches clean: dirty lines would
// be written back to HBM during the next kernel and steal its bandwidth.  The
// store only keeps the loads alive; its condition (all four words of the XOR
// equal to ~salt) does not hold on zeroed memory and practically never on
// other contents, and the buffer is scratch either way.
__global__ __launch_bounds__(256) void cache_flush_kernel(uint4* __restrict__ buf, uint64_t n16, uint32_t salt) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    const uint4 x = buf[i];
    acc.x ^= x.x;
    acc.y ^= x.y;
    acc.z ^= x.z;
    acc.w ^= x.w;
  }
  const uint32_t m = ~salt;
  if (acc.x == m && acc.y == m && acc.z == m && acc.w == m && n16) buf[0] = acc;
}

hipError_t launch_beta_read(const void* buf, uint64_t bytes, uint32_t grid, uint32_t block, int unroll,
                            uint64_t* sink, hipStream_t st) {
  const uint4* b = static_cast<const uint4*>(buf);
  const uint64_t n16 = bytes / 16u;
  switch (unroll) {
    case 1: hipLaunchKernelGGL(beta_read_kernel<1>, dim3(grid), dim3(block), 0, st, b, n16, sink); break;
    case 2: hipLaunchKernelGGL(beta_read_kernel<2>, dim3(grid), dim3(block), 0, st, b, n16, sink); break;
    case 4: hipLaunchKernelGGL(beta_read_kernel<4>, dim3(grid), dim3(block), 0, st, b, n16, sink); break;
    case 8: hipLaunchKernelGGL(beta_read_kernel<8>, dim3(grid), dim3(block), 0, st, b, n16, sink); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beta_triad(float* a, const float* b, const float* c, float s, uint64_t n, uint32_t grid,
                             hipStream_t st) {
  hipLaunchKernelGGL(beta_triad_kernel, dim3(grid), dim3(256), 0, st, reinterpret_cast<float4*>(a),
                     reinterpret_cast<const float4*>(b), reinterpret_cast<const float4*>(c), s, n / 4u);
  return hipGetLastError();
}

hipError_t launch_cache_flush(void* buf, uint64_t bytes, uint32_t grid, uint32_t salt, hipStream_t st) {
  hipLaunchKernelGGL(cache_flush_kernel, dim3(grid), dim3(256), 0, st, static_cast<uint4*>(buf), bytes / 16u, salt);
  return hipGetLastError();
}

}  // namespace scan_dev
