// Host-callable launchers for every kernel instantiation, and the per-width
// pick functions that the dispatch code looks up at run time.
#pragma once

#include "scan_kernels.h"

namespace scan_dev {

// Launch a kernel instance; with occ != nullptr only report how many
// work-groups of `block` threads fit on one compute unit.
using LaunchFn = hipError_t (*)(const Params&, uint32_t grid, uint32_t block, hipStream_t stream, int* occ);

// Whether a kernel holds no static LDS, so that its dynamic LDS starts at
// address 0 (the dictionary kernels address their entries from 0, see
// dict_at).  Checked once per kernel.
template <typename K>
inline hipError_t lds_starts_at_zero(K kern) {
  hipFuncAttributes fa;
  const hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern));
  if (e != hipSuccess) return e;
  return fa.sharedSizeBytes == 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

template <typename K>
inline hipError_t launch_kernel(K kern, bool& attr_done, const Params& p, uint32_t grid, uint32_t block,
                                uint32_t lds, hipStream_t st, int* occ) {
  if (lds > 65536u && !attr_done) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kern, (int)block, lds);
  void* args[] = {const_cast<Params*>(&p)};
  return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(block), args, lds, st);
}

template <int B, int DEC, int MODE, int ENC, int PF, int STEP = STEP_DEFAULT>
hipError_t launch_code(const Params& p, uint32_t grid, uint32_t block, hipStream_t st, int* occ) {
  static bool attr = false;
  if constexpr (ENC == ENC_DICT) {
    static const hipError_t lds0 = lds_starts_at_zero(code_scan<B, DEC, MODE, ENC, PF, STEP>);
    if (lds0 != hipSuccess) return lds0;
  }
  return launch_kernel(code_scan<B, DEC, MODE, ENC, PF, STEP>, attr, p, grid, block,
                       code_scan_lds<B, DEC, MODE, ENC>(block / 64u), st, occ);
}

// The alternative step depth exists for the register decoders' branch-free
// frame-of-reference kernels without block references, and for the
// row-major direct branch-free dictionary kernels.
template <int B, int DEC>
LaunchFn pick_code_alt(int enc, int mode, int pf) {
  if constexpr (DEC == DEC_RM_DIRECT || DEC == DEC_LI) {
    if (enc == ENC_FOR && mode == MODE_BF) {
      if (pf == PF_LO0) return &launch_code<B, DEC, MODE_BF, ENC_FOR, PF_LO0, STEP_ALT>;
      if (pf == PF_RANGE) return &launch_code<B, DEC, MODE_BF, ENC_FOR, PF_RANGE, STEP_ALT>;
    }
  }
  if constexpr (DEC == DEC_RM_DIRECT) {
    if (enc == ENC_DICT && mode == MODE_BF && pf == PF_RANGE)
      return &launch_code<B, DEC, MODE_BF, ENC_DICT, PF_RANGE, STEP_ALT>;
  }
  return nullptr;
}

template <int B, int DEC, int MODE>
hipError_t launch_delta(const Params& p, uint32_t grid, uint32_t block, hipStream_t st, int* occ) {
  static bool attr = false;
  return launch_kernel(delta_scan<B, DEC, MODE>, attr, p, grid, block, delta_scan_lds<B, DEC, MODE>(block / 64u), st,
                       occ);
}

template <int B, int DEC, int MODE, int ENC>
LaunchFn pick_pf(int pf) {
  if (pf == PF_REFS) return &launch_code<B, DEC, MODE, ENC, PF_REFS>;
  if (pf == PF_LO0) return &launch_code<B, DEC, MODE, ENC, PF_LO0>;
  return &launch_code<B, DEC, MODE, ENC, PF_RANGE>;
}

// FOR / DICT launcher for width B and decoder DEC; nullptr where the
// combination does not exist (lane-interleaved and byte-aligned are FOR only;
// byte-aligned needs B in {8, 16, 32}; dictionaries use one code range).
template <int B, int DEC>
LaunchFn pick_code(int enc, int mode, int pf) {
  if constexpr (DEC == DEC_BYTES && !(B == 8 || B == 16 || B == 32)) {
    return nullptr;
  } else {
    if (enc == ENC_FOR)
      return mode == MODE_BF ? pick_pf<B, DEC, MODE_BF, ENC_FOR>(pf) : pick_pf<B, DEC, MODE_SV, ENC_FOR>(pf);
    if constexpr (DEC == DEC_RM_LDS || DEC == DEC_RM_DIRECT) {
      if (enc == ENC_DICT && pf == PF_RANGE)
        return mode == MODE_BF ? &launch_code<B, DEC, MODE_BF, ENC_DICT, PF_RANGE>
                               : &launch_code<B, DEC, MODE_SV, ENC_DICT, PF_RANGE>;
    }
    return nullptr;
  }
}

template <int B, int DEC>
LaunchFn pick_delta(int mode) {
  return mode == MODE_BF ? &launch_delta<B, DEC, MODE_BF> : &launch_delta<B, DEC, MODE_SV>;
}

// Defined in the k_*.hip instantiation units (widths 1-4, 5-8, 9-16, 17-32).
LaunchFn code_fn_rm_lds_a(int enc, int mode, int pf, int b);
LaunchFn code_fn_rm_lds_b(int enc, int mode, int pf, int b);
LaunchFn code_fn_rm_lds_c(int enc, int mode, int pf, int b);
LaunchFn code_fn_rm_lds_d(int enc, int mode, int pf, int b);
LaunchFn code_fn_rm_direct_a(int enc, int mode, int pf, int b);
LaunchFn code_fn_rm_direct_b(int enc, int mode, int pf, int b);
LaunchFn code_fn_rm_direct_c(int enc, int mode, int pf, int b);
LaunchFn code_fn_rm_direct_d(int enc, int mode, int pf, int b);
LaunchFn code_fn_li_a(int enc, int mode, int pf, int b);
LaunchFn code_fn_li_b(int enc, int mode, int pf, int b);
LaunchFn code_fn_li_c(int enc, int mode, int pf, int b);
LaunchFn code_fn_li_d(int enc, int mode, int pf, int b);
LaunchFn code_fn_bytes(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_rm_direct_a(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_rm_direct_b(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_rm_direct_c(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_rm_direct_d(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_li_a(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_li_b(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_li_c(int enc, int mode, int pf, int b);
LaunchFn code_fn_alt_li_d(int enc, int mode, int pf, int b);
LaunchFn delta_fn_rm_lds_a(int mode, int b);
LaunchFn delta_fn_rm_lds_b(int mode, int b);
LaunchFn delta_fn_rm_lds_c(int mode, int b);
LaunchFn delta_fn_rm_lds_d(int mode, int b);
LaunchFn delta_fn_rm_direct_a(int mode, int b);
LaunchFn delta_fn_rm_direct_b(int mode, int b);
LaunchFn delta_fn_rm_direct_c(int mode, int b);
LaunchFn delta_fn_rm_direct_d(int mode, int b);

}  // namespace scan_dev

#define SCAN_WIDTHS_1_4(F) F(1) F(2) F(3) F(4)
#define SCAN_WIDTHS_5_8(F) F(5) F(6) F(7) F(8)
#define SCAN_WIDTHS_9_16(F) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16)
#define SCAN_WIDTHS_17_32(F) F(17) F(18) F(19) F(20) F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30) F(31) F(32)
