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

// Block k (32 b words) of a row-major payload into the wavefront's LDS slot
// `st` with direct global-to-LDS loads: 8 b pieces of 16 bytes, at most four
// per lane, piece i = lane + 64 j landing at byte 1024 j + 16 lane of the slot
// (the load's lane layout), all in flight together and none through
// registers; the wait after them makes the block visible to the wavefront.
__device__ __forceinline__ void stage_rt_block(uint32_t* st, const uint32_t* payload, uint32_t b, uint64_t k,
                                               uint32_t lane) {
  typedef __attribute__((address_space(1))) const void GlobalV;
  typedef __attribute__((address_space(3))) void LdsV;
  const uint32_t words = 32u * b, pieces = words / 4u;
  const uint32_t* src = payload + k * words;
  __builtin_amdgcn_s_waitcnt(0);  // the slot's earlier reads have returned
#pragma unroll
  for (uint32_t j = 0; j < 4u; ++j) {
    if (64u * j >= pieces) break;  // uniform
    if (lane + 64u * j < pieces)
      __builtin_amdgcn_global_load_lds((GlobalV*)(src + 4u * (lane + 64u * j)), (LdsV*)(st + 256u * j), 16u, 0, 0);
  }
  st[words] = 0u;  // every lane writes the same pad word
  __builtin_amdgcn_s_waitcnt(0);  // every piece is in LDS
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
