"""ctypes declarations of the C ABI in include/scan.h (argument marshalling only).

The shared library is built in-tree by ``build.py`` into ``libscan.so``.
Loading fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscan.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "scan.h")

# status codes
SCAN_OK, SCAN_EINVAL, SCAN_ENOMEM, SCAN_EDEVICE, SCAN_EUNSUPPORTED, SCAN_EBUSY = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "SCAN_OK", -1: "SCAN_EINVAL", -2: "SCAN_ENOMEM", -3: "SCAN_EDEVICE",
                -4: "SCAN_EUNSUPPORTED", -5: "SCAN_EBUSY"}
ENC_FOR, ENC_DELTA, ENC_DICT = 0, 1, 2
LAYOUT_RM, LAYOUT_LI = 0, 1
DEC_RM_LDS, DEC_RM_DIRECT, DEC_LI, DEC_BYTES = 0, 1, 2, 3
PRED_BF, PRED_SV = 0, 1
ALL_MATCH = 16
STRAT_AUTO = -1
AGG_COUNT, AGG_SUM = 1, 2


def strategy(dec: int, sv: int = 0, zm: int = 0, am: int = 0) -> int:
    return dec | (sv << 2) | (zm << 3) | (am << 4)


def strategy_name(s: int) -> str:
    if s < 0:
        return "auto"
    dec = ("rm_lds", "rm_direct", "li", "bytes")[s & 3]
    name = "%s/%s/%s" % (dec, "sv" if (s >> 2) & 1 else "bf", "zm" if (s >> 3) & 1 else "nozm")
    return name + ("/am" if (s >> 4) & 1 else "")


class ScanColumn(ctypes.Structure):
    _fields_ = [("payload", ctypes.c_void_p), ("block_ref", ctypes.c_void_p),
                ("block_base", ctypes.c_void_p), ("dict", ctypes.c_void_p),
                ("dict_len", ctypes.c_uint32), ("layout", ctypes.c_uint32),
                ("zone_min", ctypes.c_void_p), ("zone_max", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("block_sum", ctypes.c_void_p)]


class ScanPredicate(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int64), ("hi", ctypes.c_int64)]


class ScanResult(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("sum", ctypes.c_int64),
                ("blocks_read", ctypes.c_uint64), ("blocks_total", ctypes.c_uint64),
                ("strategy_used", ctypes.c_int32), ("status", ctypes.c_int32)]

    def as_dict(self):
        return {"count": int(self.count), "sum": int(self.sum), "blocks_read": int(self.blocks_read),
                "blocks_total": int(self.blocks_total), "strategy_used": int(self.strategy_used),
                "status": int(self.status)}


class ScanItem(ctypes.Structure):
    _fields_ = [("col", ScanColumn), ("enc", ctypes.c_int32), ("b", ctypes.c_uint32),
                ("pred", ScanPredicate), ("agg", ctypes.c_uint32), ("strategy", ctypes.c_int32)]


class ScanTune(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("window_blocks", ctypes.c_int32), ("depth", ctypes.c_int32)]


class ScanBatchStats(ctypes.Structure):
    _fields_ = [("captured", ctypes.c_int32), ("kernels", ctypes.c_uint32), ("class_mask", ctypes.c_uint32),
                ("work_items", ctypes.c_uint32), ("pruned", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ScanRleColumn(ctypes.Structure):
    _fields_ = [("run_value", ctypes.c_void_p), ("run_len", ctypes.c_void_p), ("block_run", ctypes.c_void_p),
                ("zone_min", ctypes.c_void_p), ("zone_max", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class ScanTableColumn(ctypes.Structure):
    _fields_ = [("col", ScanColumn), ("enc", ctypes.c_int32), ("b", ctypes.c_uint32)]


class ScanQuery(ctypes.Structure):
    _fields_ = [("n_filters", ctypes.c_uint32), ("filter_col", ctypes.c_uint32 * 3),
                ("filter", ScanPredicate * 3), ("sum_col", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ScanQueryResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("count", ctypes.c_uint64), ("sum", ctypes.c_int64),
                ("blocks_read", ctypes.c_uint64), ("submit_us", ctypes.c_double), ("done_us", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"ticket": int(self.ticket), "count": int(self.count), "sum": int(self.sum),
                "blocks_read": int(self.blocks_read), "submit_us": float(self.submit_us),
                "done_us": float(self.done_us), "status": int(self.status)}


class ScanServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("n_streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("batch_window_us", ctypes.c_uint32),
                ("window_blocks", ctypes.c_uint32), ("wgs_per_cu", ctypes.c_uint32),
                ("kernel", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_vp, _u64, _u32, _i32, _i64, _f32 = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_float)
_P = ctypes.POINTER

SIGNATURES = {
    "scan_create": (_i32, [_P(_vp), ctypes.c_int, _vp]),
    "scan_set_stream": (_i32, [_vp, _vp]),
    "scan_destroy": (None, [_vp]),
    "scan_last_error": (ctypes.c_char_p, [_vp]),
    "scan_device_cus": (ctypes.c_int, [_vp]),
    "scan_run": (_i32, [_vp, _P(ScanColumn), _i32, _u32, _P(ScanPredicate), _u32, _i32, _P(ScanResult)]),
    "scan_run_async": (_i32, [_vp, _P(ScanItem), _vp]),
    "scan_sync": (_i32, [_vp]),
    "scan_run_static": (_i32, [_P(ScanItem), _vp, _vp]),
    "scan_set_tune": (_i32, [_vp, _i32, _u32, _i32, _P(ScanTune)]),
    "scan_get_tune": (_i32, [_vp, _i32, _u32, _i32, _P(ScanTune)]),
    "scan_autotune": (_i32, [_vp, _P(ScanColumn), _i32, _u32, _P(ScanPredicate), _i32, _i32, _P(ScanTune),
                             _P(ctypes.c_float)]),
    "scan_tune_save": (_i32, [_vp, ctypes.c_char_p]),
    "scan_tune_load": (_i32, [_vp, ctypes.c_char_p]),
    "scan_run_rle": (_i32, [_vp, _P(ScanRleColumn), _P(ScanPredicate), _u32, _P(ScanResult)]),
    "scan_run_rle_async": (_i32, [_vp, _P(ScanRleColumn), _P(ScanPredicate), _u32, _vp]),
    "scan_rle_encode": (_i32, [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _P(_u64)]),
    "scan_select": (_i32, [_vp, _P(ScanColumn), _i32, _u32, _P(ScanPredicate), _u32, _vp, _u64, _P(_u64)]),
    "scan_refine": (_i32, [_vp, _P(ScanColumn), _i32, _u32, _P(ScanPredicate), _vp, _u64, _vp, _P(_u64)]),
    "scan_gather": (_i32, [_vp, _P(ScanColumn), _i32, _u32, _vp, _u64, _vp]),
    "scan_batch_prepare": (_i32, [_vp, _P(ScanItem), ctypes.c_size_t, _P(_u64)]),
    "scan_batch_replay": (_i32, [_vp, _u64, _P(ScanResult)]),
    "scan_batch_release": (_i32, [_vp, _u64]),
    "scan_batch_run": (_i32, [_vp, _P(ScanItem), ctypes.c_size_t, _P(ScanResult)]),
    "scan_batch_set_tune": (_i32, [_vp, _P(ScanTune)]),
    "scan_batch_set_graph": (_i32, [_vp, _i32]),
    "scan_batch_autotune": (_i32, [_vp, _P(ScanItem), ctypes.c_size_t, _i32, _P(ScanTune), _P(ctypes.c_float)]),
    "scan_batch_info": (_i32, [_vp, _u64, _P(ScanBatchStats)]),
    "scan_batch_set_class_cost": (_i32, [_vp, _f32]),
    "scan_batch_set_order": (_i32, [_vp, _i32]),
    "scan_mlp_param_count": (ctypes.c_int, []),
    "scan_selector_set": (_i32, [_vp, _vp, ctypes.c_size_t]),
    "scan_selector_clear": (_i32, [_vp]),
    "scan_selector_loaded": (ctypes.c_int, [_vp]),
    "scan_selector_load": (_i32, [_vp, ctypes.c_char_p]),
    "scan_selector_save": (_i32, [_vp, ctypes.c_char_p]),
    "scan_selector_set_margin": (_i32, [_vp, _f32]),
    "scan_features": (_i32, [_vp, _P(ScanItem), ctypes.c_size_t, _vp]),
    "scan_mlp_forward": (_i32, [_vp, _vp, _vp, _u32, _vp]),
    "scan_mlp_loss_grad": (_i32, [_vp, _vp, _vp, _vp, _vp, _u32, _f32, _vp, _vp]),
    "scan_adam_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _u32, _i32, _f32, _f32, _f32, _f32]),
    "scan_table_create": (_i32, [_vp, _P(ScanTableColumn), _u32, _P(_vp)]),
    "scan_table_destroy": (None, [_vp]),
    "scan_query_run": (_i32, [_vp, _vp, _P(ScanQuery), ctypes.c_size_t, _P(ScanQueryResult)]),
    "scan_query_set_tune": (_i32, [_vp, _i32, _i32]),
    "scan_query_set_kernel": (_i32, [_vp, _i32]),
    "scan_server_create": (_i32, [_vp, _vp, _P(ScanServerConfig), _P(_vp)]),
    "scan_server_submit": (_i32, [_vp, _P(ScanQuery), _P(_u64)]),
    "scan_server_poll": (_i32, [_vp, _P(ScanQueryResult), ctypes.c_size_t, _P(ctypes.c_size_t), _u32]),
    "scan_server_stats": (_i32, [_vp, _P(_u64)]),
    "scan_server_clock_us": (ctypes.c_double, []),
    "scan_server_destroy": (None, [_vp]),
    "scan_serve_simulate": (_i32, [_P(ScanServerConfig), _P(ctypes.c_double), ctypes.c_size_t, ctypes.c_double,
                                   ctypes.c_double, _P(ctypes.c_double), _P(ctypes.c_double), _P(_i32), _P(_u64)]),
    "scan_payload_words": (_u64, [_u64, _u32]),
    "scan_encode_for": (_i32, [_vp, _u64, _u32, _u32, _i32, _vp, _vp, _vp, _vp]),
    "scan_encode_delta": (_i32, [_vp, _u64, _u32, _vp, _vp, _vp, _vp]),
    "scan_encode_dict": (_i32, [_vp, _u64, _u32, _u32, _vp, _vp, _vp]),
    "scan_block_sums": (_i32, [_i32, _vp, _u64, _vp, _u32, _vp]),
    "scan_beta_read": (_i32, [_vp, _vp, _u64, _i32, _i32, _i32, _vp]),
    "scan_beta_triad": (_i32, [_vp, _vp, _vp, _vp, _f32, _u64]),
    "scan_cache_flush": (_i32, [_vp, _vp, _u64]),
}

_lib = None


class ScanError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def header_functions():
    """Every function the public header declares (name list)."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scan_[a-z0-9_]+)\s*\(", text)) - {"scan_status"})


def load():
    """Load libscan.so (built by build.py).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libscan.so is not built: run `python paper_2606_22423_amd/build.py` "
                               "(or __graft_entry__.build()); there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def register(name, restype, argtypes):
    """Declare an additional entry point (used by the batch/selector/serving modules)."""
    SIGNATURES[name] = (restype, argtypes)
    if _lib is not None:
        f = getattr(_lib, name)
        f.restype = restype
        f.argtypes = argtypes
