"""CPU oracle for the fused columnar scan -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it, and
the two share no code: the oracle's C core (``scan_oracle.c``) and its fp64
MLP reference (``mlp.py``) are written from the paper's definitions alone.

Functions take and return numpy arrays; each one cites the passage it follows
in ``scan_oracle.c``'s header.  Every function here is pinned by a CPU test
against something other than itself (see tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scan_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

L = 1024


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("sum", ctypes.c_int64),
                ("blocks_read", ctypes.c_uint64), ("blocks_total", ctypes.c_uint64),
                ("sum_overflow", ctypes.c_int32)]


class _Column(ctypes.Structure):
    _fields_ = [("enc", ctypes.c_int32), ("b", ctypes.c_uint32), ("payload", ctypes.c_void_p),
                ("refs", ctypes.c_void_p), ("dict", ctypes.c_void_p), ("m", ctypes.c_uint32)]


@dataclass(frozen=True)
class ScanResult:
    count: int
    sum: int
    blocks_read: int
    blocks_total: int
    sum_overflow: bool


def build(force: bool = False) -> str:
    """Compile the oracle's C core with gcc."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        vp, u64, u32, i32, i64 = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                  ctypes.c_int64)
        rp = ctypes.POINTER(_Result)
        sig = {
            "orc_pack_rm": [vp, u64, u32, vp],
            "orc_pack_li": [vp, u64, u32, vp],
            "orc_unpack": [vp, u64, u32, i32, vp],
            "orc_for_encode": [vp, u64, u32, i32, vp, vp],
            "orc_delta_encode": [vp, u64, u32, vp, vp],
            "orc_delta_decode": [vp, vp, u64, vp],
            "orc_dict_encode": [vp, u64, vp, u32, vp],
            "orc_zonemap_u32": [vp, u64, vp, vp],
            "orc_zonemap_i64": [vp, u64, vp, vp],
            "orc_scan_for": [vp, vp, u64, u32, i32, i64, i64, i32, rp],
            "orc_scan_delta": [vp, vp, u64, u32, i64, i64, i32, rp],
            "orc_scan_dict": [vp, vp, u32, u64, u32, i64, i64, i32, rp],
            "orc_count_sum_u32": [vp, u64, i64, i64, rp],
            "orc_count_sum_i64": [vp, u64, i64, i64, rp],
            "orc_query": [ctypes.POINTER(_Column), u64, i32, vp, vp, vp, i32, rp],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        for name, args in {"orc_select": [i32, vp, vp, vp, u64, u32, i32, i64, i64, vp, u64],
                           "orc_refine": [i32, vp, vp, vp, u32, i32, i64, i64, vp, u64, vp]}.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int64
        lib.orc_gather.argtypes = [i32, vp, vp, vp, u32, i32, vp, u64, vp]
        lib.orc_gather.restype = ctypes.c_int
        lib.orc_rle_encode.argtypes = [vp, u64, vp, vp, vp]
        lib.orc_rle_encode.restype = ctypes.c_int64
        lib.orc_rle_decode.argtypes = [vp, vp, vp, u64, vp]
        lib.orc_rle_decode.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s failed (code %d)" % (what, rc))


def _res(r: _Result) -> ScanResult:
    return ScanResult(int(r.count), int(r.sum), int(r.blocks_read), int(r.blocks_total),
                      bool(r.sum_overflow))


def nblocks(n: int) -> int:
    return (n + L - 1) // L


def payload_words(n: int, b: int) -> int:
    return nblocks(n) * 32 * b


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# ------------------------------------------------------------------ packing
def pack_rm(codes, b: int) -> np.ndarray:
    codes = _u32(codes)
    out = np.empty(payload_words(len(codes), b), dtype=np.uint32)
    _check(_load().orc_pack_rm(_ptr(codes), len(codes), b, _ptr(out)), "pack_rm")
    return out


def pack_li(codes, b: int) -> np.ndarray:
    codes = _u32(codes)
    out = np.empty(payload_words(len(codes), b), dtype=np.uint32)
    _check(_load().orc_pack_li(_ptr(codes), len(codes), b, _ptr(out)), "pack_li")
    return out


def unpack(words, n: int, b: int, layout: int = 0) -> np.ndarray:
    words = _u32(words)
    if len(words) < payload_words(n, b):
        raise ValueError("payload too short")
    out = np.empty(n, dtype=np.uint32)
    _check(_load().orc_unpack(_ptr(words), n, b, layout, _ptr(out)), "unpack")
    return out


# ---------------------------------------------------------------- encodings
def for_encode(v, b: int, policy: int = 0):
    """(refs, codes): policy 0 = reference 0, policy 1 = per-block minimum."""
    v = _u32(v)
    refs = np.empty(nblocks(len(v)), dtype=np.uint32)
    codes = np.empty(len(v), dtype=np.uint32)
    _check(_load().orc_for_encode(_ptr(v), len(v), b, policy, _ptr(refs), _ptr(codes)), "for_encode")
    return refs, codes


def delta_encode(v, b: int):
    v = _i64(v)
    bases = np.empty(nblocks(len(v)), dtype=np.int64)
    codes = np.empty(len(v), dtype=np.uint32)
    _check(_load().orc_delta_encode(_ptr(v), len(v), b, _ptr(bases), _ptr(codes)), "delta_encode")
    return bases, codes


def delta_decode(codes, bases) -> np.ndarray:
    codes, bases = _u32(codes), _i64(bases)
    out = np.empty(len(codes), dtype=np.int64)
    _check(_load().orc_delta_decode(_ptr(codes), _ptr(bases), len(codes), _ptr(out)), "delta_decode")
    return out


def dict_encode(v, dct) -> np.ndarray:
    v, dct = _i64(v), _i64(dct)
    out = np.empty(len(v), dtype=np.uint32)
    _check(_load().orc_dict_encode(_ptr(v), len(v), _ptr(dct), len(dct), _ptr(out)), "dict_encode")
    return out


def zonemap_u32(v):
    v = _u32(v)
    mn = np.empty(nblocks(len(v)), dtype=np.uint32)
    mx = np.empty_like(mn)
    _load().orc_zonemap_u32(_ptr(v), len(v), _ptr(mn), _ptr(mx))
    return mn, mx


def zonemap_i64(v):
    v = _i64(v)
    mn = np.empty(nblocks(len(v)), dtype=np.int64)
    mx = np.empty_like(mn)
    _load().orc_zonemap_i64(_ptr(v), len(v), _ptr(mn), _ptr(mx))
    return mn, mx


# -------------------------------------------------------------------- scans
def _flags(zone_maps: bool, all_match: bool) -> int:
    """Bit 0 zone maps, bit 1 the all-match shortcut (meaningful with zone maps)."""
    return int(bool(zone_maps)) | (int(bool(all_match)) << 1)


def scan_for(payload, n: int, b: int, lo: int, hi: int, refs=None, layout: int = 0,
             zone_maps: bool = False, all_match: bool = False) -> ScanResult:
    payload = _u32(payload)
    refs = None if refs is None else _u32(refs)
    r = _Result()
    _check(_load().orc_scan_for(_ptr(payload), _ptr(refs), n, b, layout, lo, hi, _flags(zone_maps, all_match),
                                ctypes.byref(r)), "scan_for")
    return _res(r)


def scan_delta(payload, bases, n: int, b: int, lo: int, hi: int, zone_maps: bool = False,
               all_match: bool = False) -> ScanResult:
    payload, bases = _u32(payload), _i64(bases)
    r = _Result()
    _check(_load().orc_scan_delta(_ptr(payload), _ptr(bases), n, b, lo, hi, _flags(zone_maps, all_match),
                                  ctypes.byref(r)), "scan_delta")
    return _res(r)


def scan_dict(payload, dct, n: int, b: int, lo: int, hi: int, zone_maps: bool = False,
              all_match: bool = False) -> ScanResult:
    payload, dct = _u32(payload), _i64(dct)
    r = _Result()
    _check(_load().orc_scan_dict(_ptr(payload), _ptr(dct), len(dct), n, b, lo, hi, _flags(zone_maps, all_match),
                                 ctypes.byref(r)), "scan_dict")
    return _res(r)


def count_sum(values, lo: int, hi: int) -> ScanResult:
    """The plain definition on raw (unpacked) values."""
    r = _Result()
    if values.dtype == np.int64:
        v = _i64(values)
        _load().orc_count_sum_i64(_ptr(v), len(v), lo, hi, ctypes.byref(r))
    else:
        v = _u32(values)
        _load().orc_count_sum_u32(_ptr(v), len(v), lo, hi, ctypes.byref(r))
    return _res(r)


def query(columns, n: int, filters, sum_col: int) -> ScanResult:
    """Conjunctive range filter over packed table columns plus SUM of another.

    columns: list of dicts {enc: 0|2, b, payload, refs (or None), dict (or None)};
    filters: [(column index, lo, hi)]."""
    keep = []
    arr = (_Column * len(columns))()
    for i, c in enumerate(columns):
        p = _u32(c["payload"])
        refs = None if c.get("refs") is None else _u32(c["refs"])
        d = None if c.get("dict") is None else _i64(c["dict"])
        keep += [p, refs, d]
        arr[i] = _Column(int(c["enc"]), int(c["b"]), _ptr(p), _ptr(refs), _ptr(d),
                         0 if d is None else len(d))
    fcol = np.array([f[0] for f in filters], dtype=np.int32)
    flo = np.array([f[1] for f in filters], dtype=np.int64)
    fhi = np.array([f[2] for f in filters], dtype=np.int64)
    r = _Result()
    _check(_load().orc_query(arr, n, len(filters), _ptr(fcol), _ptr(flo), _ptr(fhi), sum_col,
                             ctypes.byref(r)), "query")
    return _res(r)


# ------------------------------------------------------ materializing select
def select(enc: int, payload, n: int, b: int, lo: int, hi: int, refs=None, dct=None, layout: int = 0) -> np.ndarray:
    """Ascending positions i with lo <= v_i < hi (frame of reference: enc 0; dictionary: enc 2)."""
    payload = _u32(payload)
    refs = None if refs is None else _u32(refs)
    dct = None if dct is None else _i64(dct)
    cnt = _load().orc_select(enc, _ptr(payload), _ptr(refs), _ptr(dct), n, b, layout, lo, hi, None, 0)
    if cnt < 0:
        raise ValueError("oracle select rejected its arguments")
    out = np.zeros(max(cnt, 1), dtype=np.uint32)
    _load().orc_select(enc, _ptr(payload), _ptr(refs), _ptr(dct), n, b, layout, lo, hi, _ptr(out), cnt)
    return out[:cnt]


def refine(enc: int, payload, b: int, lo: int, hi: int, positions, refs=None, dct=None, layout: int = 0) -> np.ndarray:
    """The positions (ascending, kept in order) whose value in this column lies in [lo, hi)."""
    payload = _u32(payload)
    refs = None if refs is None else _u32(refs)
    dct = None if dct is None else _i64(dct)
    pos = _u32(positions)
    out = np.zeros(max(len(pos), 1), dtype=np.uint32)
    cnt = _load().orc_refine(enc, _ptr(payload), _ptr(refs), _ptr(dct), b, layout, lo, hi, _ptr(pos), len(pos),
                             _ptr(out))
    if cnt < 0:
        raise ValueError("oracle refine rejected its arguments")
    return out[:cnt]


def gather(enc: int, payload, b: int, positions, refs=None, dct=None, layout: int = 0) -> np.ndarray:
    """Decoded values at the positions (int64)."""
    payload = _u32(payload)
    refs = None if refs is None else _u32(refs)
    dct = None if dct is None else _i64(dct)
    pos = _u32(positions)
    out = np.zeros(max(len(pos), 1), dtype=np.int64)
    _check(_load().orc_gather(enc, _ptr(payload), _ptr(refs), _ptr(dct), b, layout, _ptr(pos), len(pos), _ptr(out)),
           "gather")
    return out[:len(pos)]


# ---------------------------------------------------------------- run length
def rle_encode(values):
    """(run values u32, run lengths u16, block run starts u64 [nb + 1]); runs stay inside 1024-value blocks."""
    v = _u32(values)
    n = len(v)
    rv = np.zeros(max(n, 1), dtype=np.uint32)
    rl = np.zeros(max(n, 1), dtype=np.uint16)
    br = np.zeros(nblocks(n) + 1, dtype=np.uint64)
    runs = _load().orc_rle_encode(_ptr(v), n, _ptr(rv), _ptr(rl), _ptr(br))
    return rv[:runs].copy(), rl[:runs].copy(), br


def rle_decode(rv, rl, br) -> np.ndarray:
    rv, br = _u32(rv), np.ascontiguousarray(br, dtype=np.uint64)
    rl = np.ascontiguousarray(rl, dtype=np.uint16)
    nb = len(br) - 1
    n = int(rl.astype(np.uint64).sum())
    out = np.zeros(max(n, 1), dtype=np.uint32)
    _check(_load().orc_rle_decode(_ptr(rv), _ptr(rl), _ptr(br), nb, _ptr(out)), "rle_decode")
    return out[:n]
