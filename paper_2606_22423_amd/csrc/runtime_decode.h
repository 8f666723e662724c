// Row-major decoding with the width known only at run time (kernels that
// mix columns of different widths in one launch): a wavefront stages one
// 1024-value block in LDS with 16-byte loads and lane l extracts values
// j = l + 64 t (t < 16) with a funnel shift whose shift amount is the same
// for every t of that lane.
#pragma once

#include "device_common.h"

namespace scan_dev {

constexpr uint32_t kRtStageWords = 32u * 32u + 4u;  // one block of b <= 32, plus the funnel's spill word

__device__ __forceinline__ uint32_t lower_bound_global(const int64_t* d, uint32_t m, int64_t x) {
  uint32_t lo = 0, e = m;
  while (lo < e) {
    const uint32_t mid = (lo + e) >> 1;
    if (d[mid] < x) lo = mid + 1u;
    else e = mid;
  }
  return lo;
}

// Block k (32 b words) of a row-major payload into the wavefront's LDS slot.
__device__ __forceinline__ void stage_rt_block(uint32_t* st, const uint32_t* payload, uint32_t b, uint64_t k,
                                               uint32_t lane) {
  const uint32_t words = 32u * b;
  const uint4* src = reinterpret_cast<const uint4*>(payload + k * words);
  uint4* dst = reinterpret_cast<uint4*>(st);
  __builtin_amdgcn_wave_barrier();
  for (uint32_t i = lane; i < words / 4u; i += 64u) dst[i] = src[i];
  st[words] = 0u;  // every lane writes the same pad word
  __builtin_amdgcn_wave_barrier();
}

// Code of value j = lane + 64 t of the staged block.
struct Extract {
  const uint32_t* sp;
  uint32_t sh, mask, step;
  __device__ __forceinline__ Extract(const uint32_t* st, uint32_t lane, uint32_t b) {
    const uint32_t bit0 = lane * b;
    sp = st + (bit0 >> 5);
    sh = bit0 & 31u;
    mask = b >= 32u ? 0xFFFFFFFFu : ((1u << b) - 1u);
    step = 2u * b;  // words between t and t + 1
  }
  __device__ __forceinline__ uint32_t operator()(uint32_t t) const {
    const uint32_t* w = sp + step * t;
    return funnel(w[1], w[0], sh) & mask;
  }
};

// Code of value i of a row-major column, read straight from global memory
// (random access: the second word is read only when the code straddles it,
// so no read passes the end of the block).
__device__ __forceinline__ uint32_t code_at(const uint32_t* payload, uint32_t b, uint64_t i) {
  const uint64_t k = i >> 10;
  const uint32_t bit = (uint32_t)(i & 1023u) * b;
  const uint32_t* w = payload + k * (32u * b) + (bit >> 5);
  const uint32_t sh = bit & 31u;
  const uint32_t mask = b >= 32u ? 0xFFFFFFFFu : ((1u << b) - 1u);
  const uint32_t hi = (sh + b > 32u) ? w[1] : 0u;
  return funnel(hi, w[0], sh) & mask;
}

}  // namespace scan_dev
