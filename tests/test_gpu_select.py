"""GPU parity of the materializing select, refinement and gather: the
position lists must equal the CPU oracle's element by element (ascending row
order), with zone maps and the all-match shortcut on or off."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2606_22423_amd import _lib, api  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def preds(v, b):
    top = 1 << b
    x = int(v[len(v) // 2])
    return [(0, top), (x, x + 1), (top // 5, top // 2), (-9, 3), (top - 2, top + 50), (6, 6), (9, 2)]


@pytest.mark.parametrize("b", [1, 5, 8, 13, 16, 24, 32])
def test_select_for_matches_oracle(ctx, b):
    for n in (1, 1023, 1025, 5 * 1024 + 77):
        raw = synth.width_values(synth.pcg32(501, b, n), b)
        for v in (raw, np.sort(raw)):
            w = oracle.pack_rm(v, b)
            col = api.encode_for(v, b)
            for lo, hi in preds(v, b):
                want = oracle.select(0, w, n, b, lo, hi)
                for zm, am in ((False, False), (True, False), (True, True)):
                    got = u32(ctx.select(col, lo, hi, zone_maps=zm, all_match=am))
                    assert np.array_equal(got, want), (b, n, lo, hi, zm, am, len(got), len(want))


def test_select_with_references_and_dictionary(ctx):
    n = 9 * 1024 + 3
    for b in (4, 12, 20):
        base = (np.arange(n) // 1024 * 1000003).astype(np.uint64)
        v = (base + synth.width_values(synth.pcg32(502, b, n), b)).astype(np.uint32)
        refs, codes = oracle.for_encode(v, b, policy=1)
        w = oracle.pack_rm(codes, b)
        col = api.encode_for(v, b, ref_policy=1)
        for lo, hi in [(int(v[100]), int(v[8000])), (0, 1 << 32), (int(v[3000]), int(v[3000]) + 1)]:
            want = oracle.select(0, w, n, b, lo, hi, refs=refs)
            assert np.array_equal(u32(ctx.select(col, lo, hi)), want), (b, lo, hi)
        m = min(1 << b, 4096)
        dct = synth.dict_entries(m, 503, b, 38)
        cds = synth.bounded(504, b, n, m).astype(np.uint32)
        w = oracle.pack_rm(cds, b)
        col = api.encode_dict(cds, b, dct)
        for lo, hi in [(int(dct[0]), int(dct[-1]) + 1), (int(dct[m // 3]), int(dct[m // 2])), (int(dct[1]) + 1, int(dct[2]))]:
            want = oracle.select(2, w, n, b, lo, hi, dct=dct)
            assert np.array_equal(u32(ctx.select(col, lo, hi)), want), ("dict", b, lo, hi)


def test_select_capacity_and_errors(ctx):
    v = synth.width_values(synth.pcg32(505, 10, 5000), 10)
    col = api.encode_for(v, 10)
    c = col.struct(True)
    pred = _lib.ScanPredicate(0, 512)
    cnt = ctypes.c_uint64()
    out = torch.empty(10, dtype=torch.int32, device="cuda")
    rc = ctx.lib.scan_select(ctx.h, ctypes.byref(c), col.enc, col.b, ctypes.byref(pred), 1, out.data_ptr(), 10,
                             ctypes.byref(cnt))
    assert rc == _lib.SCAN_ENOMEM and cnt.value == int(np.sum(v < 512))
    delta = api.encode_delta(np.cumsum(np.ones(3000, dtype=np.int64)), 2)
    with pytest.raises(_lib.ScanError):
        ctx.select(delta, 0, 10)


def test_select_into_full_capacity_buffer(ctx):
    """capacity >= n: count, scan and writes in one call with one wait; the
    same buffer reused by calls on different columns and predicates."""
    buf = torch.full((6 * 1024 + 500,), -1, dtype=torch.int32, device="cuda")
    for b, n in ((8, 6 * 1024 + 500), (17, 2 * 1024 + 9), (3, 1)):
        v = synth.width_values(synth.pcg32(511, b, n), b)
        w = oracle.pack_rm(v, b)
        col = api.encode_for(v, b)
        for lo, hi in preds(v, b):
            for zm in (False, True):
                got = u32(ctx.select(col, lo, hi, zone_maps=zm, out=buf))
                assert np.array_equal(got, oracle.select(0, w, n, b, lo, hi)), (b, n, lo, hi, zm)
    with pytest.raises(ValueError):
        ctx.select(api.encode_for(np.zeros(buf.numel() + 1, dtype=np.uint32), 1), 0, 1, out=buf)


def test_refine_and_gather_match_oracle(ctx):
    n = 12 * 1024 + 11
    a = synth.width_values(synth.pcg32(506, 12, n), 12)
    b = synth.width_values(synth.pcg32(507, 7, n), 7)
    m = 300
    dct = synth.dict_entries(m, 508, 9, 38)
    d = synth.bounded(509, 9, n, m).astype(np.uint32)
    wa, wb, wd = oracle.pack_rm(a, 12), oracle.pack_rm(b, 7), oracle.pack_rm(d, 9)
    ca, cb, cd = api.encode_for(a, 12), api.encode_for(b, 7), api.encode_dict(d, 9, dct)
    pos = ctx.select(ca, 1000, 3000)
    want = oracle.select(0, wa, n, 12, 1000, 3000)
    assert np.array_equal(u32(pos), want)
    r1 = ctx.refine(cb, 10, 90, pos)
    w1 = oracle.refine(0, wb, 7, 10, 90, want)
    assert np.array_equal(u32(r1), w1)
    r2 = ctx.refine(cd, int(dct[20]), int(dct[200]), r1)
    w2 = oracle.refine(2, wd, 9, int(dct[20]), int(dct[200]), w1, dct=dct)
    assert np.array_equal(u32(r2), w2) and len(w2) > 0
    # gathers, including an unsorted position list (refine keeps input order)
    perm = np.random.default_rng(5).permutation(want).astype(np.uint32)
    pt = torch.from_numpy(perm.view(np.int32)).cuda()
    assert np.array_equal(ctx.gather(ca, pt).cpu().numpy(), oracle.gather(0, wa, 12, perm))
    assert np.array_equal(ctx.gather(cd, pt).cpu().numpy(), oracle.gather(2, wd, 9, perm, dct=dct))
    rp = ctx.refine(cb, 10, 90, pt)
    assert np.array_equal(u32(rp), oracle.refine(0, wb, 7, 10, 90, perm))
    assert ctx.refine(cb, 5, 5, pt).numel() == 0


def test_select_large_column_properties(ctx):
    """2^24 values: count equals the scan's count, positions strictly ascending,
    and the values at a sample of positions pass while their neighbours'
    status matches the oracle."""
    n, b = 1 << 24, 16
    v = synth.config2_column(synth.config2_draws(n), b)
    col = api.encode_for(v, b)
    lo, hi = 1000, 9000
    pos = u32(ctx.select(col, lo, hi))
    r = ctx.run(col, lo, hi, _lib.strategy(_lib.DEC_RM_DIRECT))
    assert len(pos) == r["count"]
    full = u32(ctx.select(col, lo, hi, out=torch.empty(n, dtype=torch.int32, device="cuda")))
    assert np.array_equal(full, pos)
    assert np.all(np.diff(pos.astype(np.int64)) > 0)
    assert np.all((v[pos] >= lo) & (v[pos] < hi))
    assert int(v[pos].astype(np.uint64).sum()) == r["sum"]


def test_positions_past_the_column_are_ignored(ctx):
    v = synth.width_values(synth.pcg32(510, 9, 3000), 9)
    col = api.encode_for(v, 9)
    bad = torch.tensor([5, 2999, 3000, 70000, 17], dtype=torch.int32, device="cuda")
    got = ctx.gather(col, bad).cpu().numpy()
    assert got.tolist() == [int(v[5]), int(v[2999]), 0, 0, int(v[17])]
    kept = u32(ctx.refine(col, 0, 1 << 9, bad))
    assert kept.tolist() == [5, 2999, 17]
