// Instantiation unit: delta_fn_rm_lds_a (widths 1-4).
#include "launch_tables.h"

namespace scan_dev {
#define CASE(B) \
  case B:       \
    return pick_delta<B, DEC_RM_LDS>(mode);
LaunchFn delta_fn_rm_lds_a(int mode, int b) {
  switch (b) { SCAN_WIDTHS_1_4(CASE) }
  return nullptr;
}
}  // namespace scan_dev
