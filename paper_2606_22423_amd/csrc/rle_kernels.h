// Fused scan of run-length encoded columns (rle_kernels.hip).
#pragma once

#include "device_common.h"

namespace scan_dev {

struct RleParams {
  const uint32_t* run_value;
  const uint16_t* run_len;
  const uint64_t* block_run;  // nb + 1 run starts
  const uint32_t* zmin;       // zone maps of the values, or null
  const uint32_t* zmax;
  Result* out;                // device result (written whole by the launch)
  Partial* partials;          // per-work-group partials (at least grid entries)
  uint64_t nb;
  int64_t lo, hi;
  uint32_t use_zm, use_am;
  int32_t strategy_used;      // reported flags
  uint32_t empty;             // n == 0 or lo >= hi: only the cleared result is written
};

hipError_t launch_rle_scan(const RleParams& p, uint32_t grid, hipStream_t st);

}  // namespace scan_dev
