// Instantiation unit: byte-aligned widths 8, 16, 32.
#include "launch_tables.h"

namespace scan_dev {
LaunchFn code_fn_bytes(int enc, int mode, int pf, int b) {
  switch (b) {
    case 8: return pick_code<8, DEC_BYTES>(enc, mode, pf);
    case 16: return pick_code<16, DEC_BYTES>(enc, mode, pf);
    case 32: return pick_code<32, DEC_BYTES>(enc, mode, pf);
  }
  return nullptr;
}
}  // namespace scan_dev
