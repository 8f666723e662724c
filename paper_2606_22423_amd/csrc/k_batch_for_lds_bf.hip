// Instantiation unit: the batched class scan for (ENC_FOR, DEC_RM_LDS, MODE_BF).
#include "batch_kernels.h"

namespace scan_dev {
hipError_t launch_batch_for_lds_bf(const BatchArgs& a, uint32_t grid, uint32_t block, hipStream_t st, int* occ) {
  return launch_batch_class<ENC_FOR, DEC_RM_LDS, MODE_BF>(a, grid, block, st, occ);
}
}  // namespace scan_dev
