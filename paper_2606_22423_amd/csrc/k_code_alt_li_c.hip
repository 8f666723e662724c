// Instantiation unit: code_fn_alt_li_c (widths 9-16, alternative step depth).
#include "launch_tables.h"

namespace scan_dev {
#define CASE(B) \
  case B:       \
    return pick_code_alt<B, DEC_LI>(enc, mode, pf);
LaunchFn code_fn_alt_li_c(int enc, int mode, int pf, int b) {
  switch (b) { SCAN_WIDTHS_9_16(CASE) }
  return nullptr;
}
}  // namespace scan_dev
