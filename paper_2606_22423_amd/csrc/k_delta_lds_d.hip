// Instantiation unit: delta_fn_rm_lds_d (widths 17-32).
#include "launch_tables.h"

namespace scan_dev {
#define CASE(B) \
  case B:       \
    return pick_delta<B, DEC_RM_LDS>(mode);
LaunchFn delta_fn_rm_lds_d(int mode, int b) {
  switch (b) { SCAN_WIDTHS_17_32(CASE) }
  return nullptr;
}
}  // namespace scan_dev
