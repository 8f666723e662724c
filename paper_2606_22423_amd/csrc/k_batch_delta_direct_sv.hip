// Instantiation unit: the batched class scan for (ENC_DELTA, DEC_RM_DIRECT, MODE_SV).
#include "batch_kernels.h"

namespace scan_dev {
hipError_t launch_batch_delta_direct_sv(const BatchArgs& a, uint32_t grid, uint32_t block, hipStream_t st, int* occ) {
  return launch_batch_class<ENC_DELTA, DEC_RM_DIRECT, MODE_SV>(a, grid, block, st, occ);
}
}  // namespace scan_dev
