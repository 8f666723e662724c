"""Seeded synthetic inputs for the scan: random numbers and column recipes.

This package serves the tests, the oracle's callers and the benchmark alike.
It holds no part of the method's arithmetic: it never packs, decodes, filters
or aggregates a column.  It produces raw values and predicate bounds only.

The C core (``synth.c``) is built on first use with gcc into ``libsynth.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")
_lib = None

SEED_BASE = 0x5CA11  # per-configuration seed = SEED_BASE + (configuration number - 1)


def build(force: bool = False) -> str:
    """Compile the generator core with gcc (seconds)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        u64, i32, u32, vp, dbl = (ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                                  ctypes.c_double)
        lib.synth_pcg32_fill.argtypes = [u64, u64, u64, u64, vp, i32]
        lib.synth_pcg32_bounded_fill.argtypes = [u64, u64, u64, u64, u32, vp, i32]
        lib.synth_unit_fill.argtypes = [u64, u64, u64, u64, vp, i32]
        lib.synth_gauss_fill.argtypes = [u64, u64, u64, u64, dbl, vp, i32]
        lib.synth_fisher_yates.argtypes = [u64, u64, vp, u64]
        for f in (lib.synth_pcg32_fill, lib.synth_pcg32_bounded_fill, lib.synth_unit_fill,
                  lib.synth_gauss_fill, lib.synth_fisher_yates):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def pcg32(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """PCG32 outputs offset..offset+n-1 of the (seed, stream) sequence, uint32."""
    out = np.empty(int(n), dtype=np.uint32)
    _load().synth_pcg32_fill(seed, stream, offset, n, out.ctypes.data, _threads())
    return out


def bounded(seed: int, stream: int, n: int, rng: int, offset: int = 0) -> np.ndarray:
    """Lemire multiply-shift draws in [0, rng), uint32 (one PCG output each)."""
    if not 0 < rng <= 2**32 - 1:
        raise ValueError("range must be in [1, 2^32)")
    out = np.empty(int(n), dtype=np.uint32)
    _load().synth_pcg32_bounded_fill(seed, stream, offset, n, rng, out.ctypes.data, _threads())
    return out


def unit(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in (0,1)."""
    out = np.empty(int(n), dtype=np.float64)
    _load().synth_unit_fill(seed, stream, offset, n, out.ctypes.data, _threads())
    return out


def gauss(seed: int, stream: int, n: int, clip: float = 8.0, offset: int = 0) -> np.ndarray:
    """Box-Muller normals clipped to [-clip, clip] (clip <= 0 disables clipping)."""
    out = np.empty(int(n), dtype=np.float64)
    _load().synth_gauss_fill(seed, stream, offset, n, clip, out.ctypes.data, _threads())
    return out


def fisher_yates(seed: int, stream: int, n: int) -> np.ndarray:
    """A uniformly random permutation of 0..n-1 (uint32) by Fisher-Yates."""
    perm = np.arange(n, dtype=np.uint32)
    if _load().synth_fisher_yates(seed, stream, perm.ctypes.data, n) != 0:
        raise ValueError("n too large for Fisher-Yates")
    return perm


from .workloads import *  # noqa: E402,F401,F403
