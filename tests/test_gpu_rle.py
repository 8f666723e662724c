"""GPU parity of the fused run-length scan: COUNT, SUM and blocks_read equal
the oracle's plain definition on the decoded values (tolerance 0)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2606_22423_amd import _lib, api  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 1024, 1025, 9 * 1024 + 301])
def test_rle_scan_matches_oracle(ctx, n):
    rng = np.random.default_rng(n)
    cols = [np.repeat(rng.integers(0, 1 << 20, size=n // 37 + 1), 37)[:n].astype(np.uint32),   # runs across blocks
            np.sort(synth.width_values(synth.pcg32(601, 16, n), 16)),                          # clustered
            synth.width_values(synth.pcg32(602, 3, n), 3),                                     # short runs
            np.full(n, 0xFFFFFFFF, dtype=np.uint32)]                                          # one value
    for v in cols:
        w = oracle.pack_rm(v, 32)
        col = api.encode_rle(v)
        x = int(v[n // 2])
        for lo, hi in [(0, 1 << 32), (x, x + 1), (int(v.min()), int(v.max())), (-5, 1 << 40), (7, 7), (x + 1, x)]:
            for zm, am in ((False, False), (True, False), (True, True)):
                want = oracle.scan_for(w, n, 32, lo, hi, zone_maps=zm, all_match=am)
                got = ctx.run_rle(col, lo, hi, zone_maps=zm, all_match=am)
                assert (got["count"], got["sum"], got["blocks_read"], got["blocks_total"]) == \
                    (want.count, want.sum, want.blocks_read, want.blocks_total), (n, lo, hi, zm, am, got, want)


def test_rle_async_result_equals_sync(ctx):
    """The enqueued scan writes the whole 40-byte result to device memory,
    the same fields as the synchronous call, also for an empty predicate and
    a run-heavy column spanning many 64-block chunks."""
    n = 200 * 1024 + 77
    v = synth.width_values(synth.pcg32(603, 4, n), 4)          # short runs, ~n/1.1 of them
    s = np.sort(synth.width_values(synth.pcg32(604, 12, n), 12))  # clustered
    out = torch.zeros(5, dtype=torch.int64, device="cuda")
    for vals in (v, s):
        col = api.encode_rle(vals)
        w = oracle.pack_rm(vals, 32)
        for lo, hi in [(0, 1 << 32), (3, 9), (int(vals[n // 3]), int(vals[2 * n // 3])), (9, 3)]:
            for zm, am in ((False, False), (True, False), (True, True)):
                out.fill_(-1)
                ctx.run_rle_async(col, lo, hi, out, zone_maps=zm, all_match=am)
                ctx.sync()
                raw = out.cpu().numpy()
                got = (int(raw[0]) & 0xFFFFFFFFFFFFFFFF, int(raw[1]), int(raw[2]), int(raw[3]),
                       int(raw[4]) & 0xFFFFFFFF, int(raw[4]) >> 32)
                r = ctx.run_rle(col, lo, hi, zone_maps=zm, all_match=am)
                want = oracle.scan_for(w, n, 32, lo, hi, zone_maps=zm, all_match=am)
                assert got[:4] == (want.count, want.sum, want.blocks_read, want.blocks_total), (lo, hi, zm, am)
                assert got[:4] == (r["count"], r["sum"], r["blocks_read"], r["blocks_total"])
                assert got[4] == (1 if zm else 0) + (2 if zm and am else 0) and got[5] == 0


def test_rle_errors(ctx):
    col = api.encode_rle(np.arange(100, dtype=np.uint32))
    c = col.struct(True)
    r = _lib.ScanResult()
    pred = _lib.ScanPredicate(0, 5)
    import ctypes
    assert ctx.lib.scan_run_rle(ctx.h, ctypes.byref(c), ctypes.byref(pred), 4, ctypes.byref(r)) == _lib.SCAN_EINVAL
    bare = col.struct(False)
    assert ctx.lib.scan_run_rle(ctx.h, ctypes.byref(bare), ctypes.byref(pred), 1, ctypes.byref(r)) == \
        _lib.SCAN_EUNSUPPORTED
    # misaligned run arrays are refused before anything is enqueued
    off = col.struct(True)
    off.run_value = c.run_value + 4
    assert ctx.lib.scan_run_rle(ctx.h, ctypes.byref(off), ctypes.byref(pred), 0, ctypes.byref(r)) == _lib.SCAN_EINVAL
    off = col.struct(True)
    off.run_len = c.run_len + 2
    assert ctx.lib.scan_run_rle(ctx.h, ctypes.byref(off), ctypes.byref(pred), 0, ctypes.byref(r)) == _lib.SCAN_EINVAL
