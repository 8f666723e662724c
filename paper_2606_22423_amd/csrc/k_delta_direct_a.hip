// Instantiation unit: delta_fn_rm_direct_a (widths 1-4).
#include "launch_tables.h"

namespace scan_dev {
#define CASE(B) \
  case B:       \
    return pick_delta<B, DEC_RM_DIRECT>(mode);
LaunchFn delta_fn_rm_direct_a(int mode, int b) {
  switch (b) { SCAN_WIDTHS_1_4(CASE) }
  return nullptr;
}
}  // namespace scan_dev
