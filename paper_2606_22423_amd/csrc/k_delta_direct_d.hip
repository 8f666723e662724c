// Instantiation unit: delta_fn_rm_direct_d (widths 17-32).
#include "launch_tables.h"

namespace scan_dev {
#define CASE(B) \
  case B:       \
    return pick_delta<B, DEC_RM_DIRECT>(mode);
LaunchFn delta_fn_rm_direct_d(int mode, int b) {
  switch (b) { SCAN_WIDTHS_17_32(CASE) }
  return nullptr;
}
}  // namespace scan_dev
