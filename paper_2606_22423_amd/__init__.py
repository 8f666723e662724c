"""MI355X-native fused columnar scan (decode + predicate + COUNT/SUM with zone maps).

The hot path lives in libscan.so (HIP, gfx950) behind the C ABI of
include/scan.h; this package only marshals arguments (``_lib``, ``api``) and
hosts the measurement helpers (``lawfit``).
"""
from ._lib import (AGG_COUNT, AGG_SUM, DEC_BYTES, DEC_LI, DEC_RM_DIRECT, DEC_RM_LDS, ENC_DELTA, ENC_DICT,
                   ENC_FOR, LAYOUT_LI, LAYOUT_RM, PRED_BF, PRED_SV, STRAT_AUTO, ScanError, load, strategy,
                   strategy_name)

__all__ = ["AGG_COUNT", "AGG_SUM", "DEC_BYTES", "DEC_LI", "DEC_RM_DIRECT", "DEC_RM_LDS", "ENC_DELTA", "ENC_DICT",
           "ENC_FOR", "LAYOUT_LI", "LAYOUT_RM", "PRED_BF", "PRED_SV", "STRAT_AUTO", "ScanError", "load",
           "strategy", "strategy_name"]
