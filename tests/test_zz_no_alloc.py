"""GPU check of scan_run_static, the scan entry point that allocates nothing:
through the C ABI its result equals scan_run_async's (same kernels, partials
in the library's static device array instead of a context's allocation), on
consecutive calls whose second input is smaller than the first (the shared
array keeps the first call's partials), for every encoding and predicate
mode, an empty predicate and argument errors.  Tolerance 0 (integers)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2606_22423_amd import _lib, api  # noqa: E402
from paper_2606_22423_amd._lib import DEC_LI, DEC_RM_DIRECT, DEC_RM_LDS, LAYOUT_LI, strategy  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def columns(n, seed):
    """FOR (row-major and transposed), delta and dictionary columns of n values."""
    out = []
    for b in (3, 13, 27):
        v = synth.width_values(synth.pcg32(seed, b, n), b)
        out.append((api.encode_for(v, b), 0, (1 << b) // 3, b))
        out.append((api.encode_for(v, b, layout=LAYOUT_LI), (1 << b) // 5, (1 << b) // 2, b))
    d = synth.width_values(synth.pcg32(seed + 1, 9, n), 9).astype(np.int64)
    v = np.cumsum(d)
    out.append((api.encode_delta(v, 9), int(v[n // 3]), int(v[n // 2]), 9))
    m = 300
    codes = synth.width_values(synth.pcg32(seed + 2, 9, n), 9) % m
    dct = np.sort(np.unique(synth.width_values(synth.pcg32(seed + 3, 20, 4 * m), 20).astype(np.int64)))[:m]
    out.append((api.encode_dict(codes.astype(np.uint32), 9, dct), int(dct[40]), int(dct[200]), 9))
    return out


def strategies(col):
    if col.layout == LAYOUT_LI:
        decs = [DEC_LI]
    else:
        decs = [DEC_RM_LDS, DEC_RM_DIRECT]
    return [strategy(d, sv, zm) for d in decs for sv in (0, 1) for zm in (0, 1)] + [-1]


def test_static_entry_point_equals_async(ctx=None):
    c = api.Context(0)
    try:
        out_a = torch.zeros(5, dtype=torch.int64, device="cuda")
        out_s = torch.full((5,), -7, dtype=torch.int64, device="cuda")
        # two calls in a row, the second on a smaller input: a large column
        # (many work-groups) then a small one (few)
        for n, seed in ((3_000_000 + 77, 71), (5_000, 72)):
            for col, lo, hi, b in columns(n, seed):
                for s in strategies(col):
                    for plo, phi in ((lo, hi), (hi, lo)):
                        say("static scan n=%d enc=%d b=%d layout=%d strategy=%d pred=[%d,%d)" %
                            (n, col.enc, b, col.layout, s, plo, phi))
                        c.run_async(col, plo, phi, s, out_a)
                        api.run_static(col, plo, phi, s, out_s, stream=c.stream)
                        torch.cuda.synchronize()
                        a, st = out_a.cpu().tolist(), out_s.cpu().tolist()
                        assert a == st, (n, col.enc, b, s, plo, phi, a, st)
                        out_s.fill_(-7)
    finally:
        c.close()


def test_static_entry_point_errors():
    v = synth.width_values(synth.pcg32(5, 8, 4096), 8)
    col = api.encode_for(v, 8)
    out = torch.zeros(5, dtype=torch.int64, device="cuda")
    lib = _lib.load()
    it = col.item(0, 10, strategy(DEC_RM_DIRECT, 0, 0))
    it.b = 33
    import ctypes
    assert lib.scan_run_static(ctypes.byref(it), None, ctypes.c_void_p(out.data_ptr())) == _lib.SCAN_EINVAL
    it = col.item(0, 10, strategy(DEC_LI, 0, 0))  # a row-major column with the transposed decoder
    assert lib.scan_run_static(ctypes.byref(it), None, ctypes.c_void_p(out.data_ptr())) == _lib.SCAN_EUNSUPPORTED
    assert lib.scan_run_static(None, None, ctypes.c_void_p(out.data_ptr())) == _lib.SCAN_EINVAL
    it = col.item(0, 10, strategy(DEC_RM_DIRECT, 0, 0))
    assert lib.scan_run_static(ctypes.byref(it), None, None) == _lib.SCAN_EINVAL
