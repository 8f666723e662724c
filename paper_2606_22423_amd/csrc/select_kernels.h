// Materializing select, refinement and gather (select_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scan_dev {

constexpr uint32_t kScanTile = 1024;  // counts per work-group of the exclusive scan

struct SelParams {
  const uint32_t* payload;
  const uint32_t* refs;    // frame-of-reference block references, or null
  const int64_t* dict;     // dictionary entries
  const uint32_t* zmin;    // zone maps (values / codes), or null
  const uint32_t* zmax;
  const int64_t* zrange;   // device: the predicate in the zone-map / code domain (written by setup)
  uint64_t* marks;         // select: 1024-bit mark string per block, 16 words (bit l of word t: value l + 64 t)
  uint32_t* counts;        // per block (select) or per chunk of positions (refine)
  uint32_t* offsets;       // exclusive prefix of counts
  uint64_t n, nb;
  int64_t lo, hi;          // predicate on decoded values
  uint32_t b, enc, dict_len, use_zm, use_am, pad;
};

hipError_t launch_select_setup(const SelParams& p, int64_t* zrange, hipStream_t st);
hipError_t launch_select_mark(const SelParams& p, uint32_t grid, hipStream_t st);
hipError_t launch_exclusive_scan(const uint32_t* in, uint64_t m, uint32_t* out, uint32_t* tile_sums,
                                 uint32_t* total, hipStream_t st);
hipError_t launch_select_write(const SelParams& p, uint32_t* positions, uint32_t grid, hipStream_t st);
hipError_t launch_refine_mark(const SelParams& p, const uint32_t* pos, uint64_t m, uint64_t* ballots,
                              uint32_t* counts, uint32_t grid, hipStream_t st);
hipError_t launch_refine_write(const uint32_t* pos, uint64_t m, const uint64_t* ballots, const uint32_t* offsets,
                               uint32_t* out, uint32_t grid, hipStream_t st);
hipError_t launch_gather(const SelParams& p, const uint32_t* pos, uint64_t m, int64_t* values, hipStream_t st);

}  // namespace scan_dev
