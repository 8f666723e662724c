// Instantiation unit: delta_fn_rm_lds_b (widths 5-8).
#include "launch_tables.h"

namespace scan_dev {
#define CASE(B) \
  case B:       \
    return pick_delta<B, DEC_RM_LDS>(mode);
LaunchFn delta_fn_rm_lds_b(int mode, int b) {
  switch (b) { SCAN_WIDTHS_5_8(CASE) }
  return nullptr;
}
}  // namespace scan_dev
