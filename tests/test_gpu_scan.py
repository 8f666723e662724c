"""GPU parity: every scan strategy, bit-exact against the CPU oracle.

Inputs come from the shared seeded generators; the GPU reads the library
encoder's bytes, the oracle packs the same raw values itself.  Tolerance is
zero: count, sum and blocks_read are integers.
"""
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
from paper_2606_22423_amd._lib import (DEC_BYTES, DEC_LI, DEC_RM_DIRECT, DEC_RM_LDS, ENC_DELTA,  # noqa: E402
                                       ENC_DICT, ENC_FOR, LAYOUT_LI, LAYOUT_RM, strategy)


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rm_strategies(b, enc=ENC_FOR):
    decs = [DEC_RM_LDS, DEC_RM_DIRECT]
    if enc == ENC_FOR and b in (8, 16, 32):
        decs.append(DEC_BYTES)
    return [strategy(d, sv, zm) for d in decs for sv in (0, 1) for zm in (0, 1)]


LI_STRATS = [strategy(DEC_LI, sv, zm) for sv in (0, 1) for zm in (0, 1)]


def check(got, want, zm, what, want_off=None):
    """want: the oracle with zone maps on.  With zone maps off every block of a
    non-empty predicate is read, so blocks_read is the block count (0 if lo >= hi)."""
    assert (got["count"], got["sum"]) == (want.count, want.sum), (what, got, want)
    if zm:
        assert got["blocks_read"] == want.blocks_read, (what, got, want)
    elif want_off is not None:
        assert got["blocks_read"] == want_off.blocks_read, (what, got, want_off)
    assert got["blocks_total"] == want.blocks_total


def preds_for(b, v, rng):
    top = 1 << b
    x = int(v[len(v) // 2])
    out = [(0, top), (0, max(1, top // 10)), (x, x + 1), (top // 3, top // 3 + max(1, top // 7)),
           (-5, 3), (top - 1, top + 100), (5, 5), (9, 2)]
    lo, hi = sorted(int(t) for t in rng.integers(0, top + 1, size=2))
    out.append((lo, hi + 1))
    return out


def test_config1_every_strategy(ctx):
    v, lo, hi = synth.config1()
    want = oracle.scan_for(oracle.pack_rm(v, 8), len(v), 8, lo, hi, zone_maps=True)
    want_off = oracle.scan_for(oracle.pack_rm(v, 8), len(v), 8, lo, hi, zone_maps=False)
    assert want.count > 100_000
    col = api.encode_for(v, 8)
    for s in rm_strategies(8):
        say("config1 strategy", _lib.strategy_name(s))
        got = ctx.run(col, lo, hi, s)
        check(got, want, (s >> 3) & 1, s, want_off)
        assert got["strategy_used"] == s
    coli = api.encode_for(v, 8, layout=LAYOUT_LI)
    for s in LI_STRATS:
        got = ctx.run(coli, lo, hi, s)
        check(got, want, (s >> 3) & 1, s, want_off)


@pytest.mark.parametrize("b", range(1, 33))
def test_for_every_width_and_strategy(ctx, b):
    rng = np.random.default_rng(1000 + b)
    for n in (1, 1023, 1025, 5 * 1024 + 77):
        v = synth.width_values(synth.pcg32(77, b * 100 + n % 97, n), b)
        v[:2] = [0, (1 << b) - 1] if n >= 2 else v[:2]
        w_rm, w_li = oracle.pack_rm(v, b), oracle.pack_li(v, b)
        col = api.encode_for(v, b)
        coli = api.encode_for(v, b, layout=LAYOUT_LI)
        for lo, hi in preds_for(b, v, rng):
            want = oracle.scan_for(w_rm, n, b, lo, hi, zone_maps=True)
            want_off = oracle.scan_for(w_rm, n, b, lo, hi, zone_maps=False)
            want_li = oracle.scan_for(w_li, n, b, lo, hi, layout=1, zone_maps=True)
            assert (want.count, want.sum, want.blocks_read) == (want_li.count, want_li.sum, want_li.blocks_read)
            for s in rm_strategies(b):
                got = ctx.run(col, lo, hi, s)
                check(got, want, (s >> 3) & 1, (b, n, lo, hi, _lib.strategy_name(s)), want_off)
            for s in LI_STRATS:
                got = ctx.run(coli, lo, hi, s)
                check(got, want, (s >> 3) & 1, (b, n, lo, hi, _lib.strategy_name(s)))


@pytest.mark.parametrize("b", [1, 5, 12, 20, 31])
def test_for_block_references(ctx, b):
    n = 6 * 1024 + 13
    top = (1 << 32) - (1 << b)  # block bases keep every value inside u32
    base = (np.repeat(np.arange(7, dtype=np.uint64) * top // 7, 1024)[:n]).astype(np.uint64)
    v = (base + synth.width_values(synth.pcg32(5, b, n), b).astype(np.uint64)).astype(np.uint32)
    refs, codes = oracle.for_encode(v, b, policy=1)
    w = oracle.pack_rm(codes, b)
    col = api.encode_for(v, b, ref_policy=1)
    rng = np.random.default_rng(b)
    for lo, hi in [(0, 1 << 32), (int(v[3000]), int(v[3000]) + 1), (1_000_000_000, 2_500_000_000),
                   (int(v.min()), int(v.min()) + (1 << b) // 2)] + \
            [tuple(sorted(int(t) for t in rng.integers(0, 1 << 32, size=2))) for _ in range(3)]:
        want = oracle.scan_for(w, n, b, lo, hi, refs=refs, zone_maps=True)
        want_off = oracle.scan_for(w, n, b, lo, hi, refs=refs, zone_maps=False)
        for s in rm_strategies(b):
            check(ctx.run(col, lo, hi, s), want, (s >> 3) & 1, (b, lo, hi, s), want_off)


@pytest.mark.parametrize("b", list(range(1, 16)))
def test_packed_field_widths_every_code_window(ctx, b):
    """b <= 15 takes the packed-field (SWAR) path on full blocks: every code
    window [lo, hi) at b <= 4 (300 and the extremes above), on both register
    decoders, with and without block references, against the oracle.  The
    ragged last block goes through the per-code loop."""
    n = 3 * 1024 + 517
    top = 1 << b
    v = synth.width_values(synth.pcg32(7, b, n), b)
    w = oracle.pack_rm(v, b)
    col, coli = api.encode_for(v, b), api.encode_for(v, b, layout=LAYOUT_LI)
    base = (np.repeat(np.arange(4, dtype=np.uint64) * 1_000_003, 1024)[:n]).astype(np.uint64)  # u32-safe for b <= 15
    vr = (base + v.astype(np.uint64)).astype(np.uint32)
    refs, codes = oracle.for_encode(vr, b, policy=1)
    wr = oracle.pack_rm(codes, b)
    colr = api.encode_for(vr, b, ref_policy=1)
    if b <= 4:
        windows = [(lo, hi) for lo in range(top + 1) for hi in range(lo, top + 2)]
    else:
        rng = np.random.default_rng(8)
        windows = [(0, 1), (0, top), (top - 1, top), (0, top - 1), (1, top), (5, 6)] + \
            [tuple(sorted(int(t) for t in rng.integers(0, top + 1, size=2))) for _ in range(300)]
    bf = [strategy(DEC_RM_DIRECT, 0, 0), strategy(DEC_LI, 0, 0)]
    for lo, hi in windows:
        want = oracle.scan_for(w, n, b, lo, hi)
        for s, c in zip(bf, (col, coli)):
            got = ctx.run(c, lo, hi, s)
            assert (got["count"], got["sum"]) == (want.count, want.sum), (b, lo, hi, _lib.strategy_name(s))
        # the same window shifted into each block's frame (references 0, 1000003, ...)
        for k in range(4):
            rlo, rhi = lo + k * 1_000_003, hi + k * 1_000_003
            want = oracle.scan_for(wr, n, b, rlo, rhi, refs=refs)
            got = ctx.run(colr, rlo, rhi, strategy(DEC_RM_DIRECT, 0, 0))
            assert (got["count"], got["sum"]) == (want.count, want.sum), (b, rlo, rhi, "refs")


@pytest.mark.parametrize("b", [1, 2, 7, 13, 16, 17, 22, 23, 28, 32])
def test_delta_every_strategy(ctx, b):
    for n in (1, 1024, 4 * 1024 + 333):
        d = synth.width_values(synth.pcg32(31, b, n), b).astype(np.int64)
        d[0] = int(synth.pcg32(32, b, 1)[0])
        v = np.cumsum(d)
        bases, codes = oracle.delta_encode(v, b)
        w = oracle.pack_rm(codes, b)
        col = api.encode_delta(v, b)
        rng = np.random.default_rng(b * 7 + n)
        preds = [(int(v[0]), int(v[-1]) + 1), (int(v[n // 2]), int(v[n // 2]) + 1), (-(1 << 62), 1 << 62),
                 (int(v[-1]) + 1, int(v[-1]) + 5), (5, 5)]
        for _ in range(3):
            p, q = sorted(int(t) for t in rng.integers(0, n, size=2))
            preds.append((int(v[p]), int(v[q]) + 1))
        for lo, hi in preds:
            want = oracle.scan_delta(w, bases, n, b, lo, hi, zone_maps=True)
            want_off = oracle.scan_delta(w, bases, n, b, lo, hi, zone_maps=False)
            for s in rm_strategies(b, ENC_DELTA):
                check(ctx.run(col, lo, hi, s), want, (s >> 3) & 1, (b, n, lo, hi, _lib.strategy_name(s)), want_off)


@pytest.mark.parametrize("b", [1, 3, 8, 12, 13, 20, 24, 32])
def test_dict_every_strategy(ctx, b):
    m = min(1 << b, 4096)
    dct = synth.dict_entries(m, 9, b, 38)
    for n in (1, 1025, 5 * 1024 + 3):
        codes = synth.bounded(8, b, n, m)
        w = oracle.pack_rm(codes, b)
        col = api.encode_dict(codes, b, dct)
        rng = np.random.default_rng(b + n)
        preds = [(int(dct[0]), int(dct[-1]) + 1), (int(dct[m // 2]), int(dct[m // 2]) + 1),
                 (int(dct[0]) - 10, int(dct[0])), (-(1 << 62), 1 << 62)]
        if m > 2:
            preds.append((int(dct[1]) + 1, int(dct[2])))  # no entry inside: empty code range
        for _ in range(3):
            i, j = sorted(int(t) for t in rng.integers(0, m, size=2))
            preds.append((int(dct[i]), int(dct[j]) + 1))
        for lo, hi in preds:
            want = oracle.scan_dict(w, dct, n, b, lo, hi, zone_maps=True)
            want_off = oracle.scan_dict(w, dct, n, b, lo, hi, zone_maps=False)
            for s in rm_strategies(b, ENC_DICT):
                check(ctx.run(col, lo, hi, s), want, (s >> 3) & 1, (b, n, lo, hi, _lib.strategy_name(s)), want_off)


def wide_dictionary(b):
    """Sorted entries over [-2^62, 2^62): for b = 3 a hand-made one with
    windows of range 2^53 - 1 and 2^53 exactly, else stratified draws."""
    if b == 3:
        e = [-(1 << 62), -(1 << 62) + 1, -(1 << 62) + (1 << 53) - 1, -(1 << 62) + (1 << 53), 0, 5,
             (1 << 62) - 3, (1 << 62) - 1]
        return np.array(e, dtype=np.int64)
    return synth.dict_entries(min(1 << b, 4096), 17, b, 62)


@pytest.mark.parametrize("b", [3, 8, 12])
def test_dict_packed_and_wide_code_windows(ctx, b):
    """Branch-free dictionary scans carry the match count inside packed
    entries when the selected entries span less than 2^53 and compare per
    code otherwise.  Windows on both sides of that bound (for b = 3: ranges
    2^53 - 1 and 2^53 exactly), negative entries and sums that wrap mod 2^64
    match the oracle in every strategy, single scans and a batch."""
    dct = wide_dictionary(b)
    m = len(dct)
    windows = [(0, 2), (0, 3), (1, 3), (0, m - 1), (4, 5), (m // 2, m // 2)] if b == 3 else \
        [(0, 0), (5, 7), (m // 3, m // 3 + 3), (m // 3, m // 3 + 5), (0, m - 1), (m - 9, m - 1)]
    for n in (5 * 1024 + 3, 300 * 1024 + 7):
        codes = synth.bounded(31, b, n, m)
        w = oracle.pack_rm(codes, b)
        col = api.encode_dict(codes, b, dct)
        items, wants = [], []
        for i, j in windows:
            lo, hi = int(dct[i]), int(dct[j]) + 1
            want = oracle.scan_dict(w, dct, n, b, lo, hi, zone_maps=True)
            want_off = oracle.scan_dict(w, dct, n, b, lo, hi, zone_maps=False)
            for s in rm_strategies(b, ENC_DICT):
                check(ctx.run(col, lo, hi, s), want, (s >> 3) & 1, (b, n, i, j, _lib.strategy_name(s)), want_off)
                items.append(col.item(lo, hi, s))
                wants.append((want, want_off, s, (b, n, i, j)))
        for got, (want, want_off, s, what) in zip(ctx.batch_run(items), wants):
            check(got, want, (s >> 3) & 1, what + ("batch", _lib.strategy_name(s)), want_off)


def test_sorted_column_zone_maps_read_exact_blocks(ctx):
    n, nd = 1 << 22, 1 << 8  # 2^14 copies per value: 16 whole blocks each
    v = synth.config3_column(n, nd, 0).numpy().astype(np.uint32)
    col = api.encode_for(v, 16)
    for lo, hi in ((0, 1), (17, 40), (0, 256), (255, 256)):
        for s in (strategy(DEC_RM_DIRECT, 0, 1), strategy(DEC_RM_LDS, 1, 1), strategy(DEC_BYTES, 0, 1)):
            got = ctx.run(col, lo, hi, s)
            assert got["count"] == (hi - lo) << 14
            assert got["sum"] == (1 << 14) * (hi - lo) * (lo + hi - 1) // 2
            assert got["blocks_read"] == 16 * (hi - lo)


def test_edge_cases_and_errors(ctx):
    v = synth.width_values(synth.pcg32(1, 1, 5000), 7)
    col = api.encode_for(v, 7)
    nb = oracle.nblocks(5000)
    r = ctx.run(col, 9, 3, strategy(DEC_RM_DIRECT, 0, 1))
    assert (r["count"], r["sum"], r["blocks_read"]) == (0, 0, 0)
    r = ctx.run(col, 1 << 40, 1 << 41, strategy(DEC_RM_DIRECT, 0, 0))
    assert (r["count"], r["sum"], r["blocks_read"], r["blocks_total"]) == (0, 0, nb, nb)
    r = ctx.run(col, 1 << 40, 1 << 41, strategy(DEC_RM_DIRECT, 0, 1))
    assert (r["count"], r["sum"], r["blocks_read"]) == (0, 0, 0)
    empty = api.Column(ENC_FOR, 7, 0, LAYOUT_RM, col.payload)
    r = ctx.run(empty, 0, 100, strategy(DEC_RM_DIRECT, 0, 0))
    assert (r["count"], r["sum"], r["blocks_total"]) == (0, 0, 0)
    with pytest.raises(_lib.ScanError) as e:
        ctx.run(col, 0, 10, strategy(DEC_LI, 0, 0))
    assert e.value.status == _lib.SCAN_EUNSUPPORTED
    with pytest.raises(_lib.ScanError) as e:
        ctx.run(col, 0, 10, strategy(DEC_BYTES, 0, 0))
    assert e.value.status == _lib.SCAN_EUNSUPPORTED
    bad = api.Column(ENC_FOR, 7, 5000, LAYOUT_RM, col.payload[1:])  # 4-byte offset: misaligned
    with pytest.raises(_lib.ScanError) as e:
        ctx.run(bad, 0, 10, strategy(DEC_RM_DIRECT, 0, 0))
    assert e.value.status == _lib.SCAN_EINVAL
    with pytest.raises(_lib.ScanError):
        ctx.run(col, 0, 10, 99)
    dcol = api.encode_dict(np.zeros(10, dtype=np.uint32), 2, np.arange(4, dtype=np.int64))
    dcol.dct = torch.arange(5, dtype=torch.int64, device="cuda")  # 5 entries > 2^2
    with pytest.raises(_lib.ScanError) as e:
        ctx.run(dcol, 0, 3, strategy(DEC_RM_DIRECT, 0, 0))
    assert e.value.status == _lib.SCAN_EINVAL


def test_async_results_and_repeat_launches(ctx):
    v = synth.width_values(synth.pcg32(3, 3, 100_000), 11)
    col = api.encode_for(v, 11)
    preds = [(0, 100), (50, 1500), (0, 2048), (1000, 1001)]
    out = torch.zeros((len(preds) * 3, 5), dtype=torch.int64, device="cuda")
    k = 0
    for lo, hi in preds:
        for s in (strategy(DEC_RM_LDS, 0, 0), strategy(DEC_RM_DIRECT, 1, 1), strategy(DEC_RM_DIRECT, 0, 1)):
            ctx.run_async(col, lo, hi, s, out[k])
            k += 1
    ctx.sync()
    host = out.cpu()
    k = 0
    w = oracle.pack_rm(v, 11)
    for lo, hi in preds:
        want = oracle.scan_for(w, len(v), 11, lo, hi, zone_maps=True)
        for s in range(3):
            r = api.result_from_tensor(host[k])
            assert (r["count"], r["sum"]) == (want.count, want.sum)
            k += 1


def test_launch_tuning_does_not_change_results(ctx):
    """Work-group size, work-groups per CU, the window size and the step depth
    are speed knobs only."""
    n = 300 * 1024 + 999
    for b in (3, 13, 16, 32):
        v = synth.width_values(synth.pcg32(44, b, n), b)
        for layout, pack in ((LAYOUT_RM, oracle.pack_rm), (LAYOUT_LI, oracle.pack_li)):
            col = api.encode_for(v, b, layout=layout)
            for lo, hi in (((1 << b) // 5, (1 << b) // 2), (0, (1 << b) // 3)):
                want = oracle.scan_for(pack(v, b), n, b, lo, hi, layout=layout, zone_maps=True)
                decs = (DEC_LI,) if layout == LAYOUT_LI else (DEC_RM_DIRECT, DEC_RM_LDS)
                for s in [strategy(d, m, z) for d in decs for m, z in ((0, 1), (1, 0), (0, 0))]:
                    for wg, per_cu, win, depth in ((64, 1, 1, 1), (128, 3, 5, 0), (256, 0, 64, 1), (192, 2, 0, 1),
                                                   (0, 0, 0, 1)):
                        ctx.set_tune(ENC_FOR, b, s, wg, per_cu, win, depth)
                        got = ctx.run(col, lo, hi, s)
                        case = (b, layout, s, wg, per_cu, win, depth, lo, hi)
                        assert (got["count"], got["sum"]) == (want.count, want.sum), case
                        if (s >> 3) & 1:
                            assert got["blocks_read"] == want.blocks_read, case
                    ctx.set_tune(ENC_FOR, b, s, 0, 0, 0, 0)


@pytest.mark.parametrize("b", [3, 8, 12, 17])
def test_dict_launch_tuning_does_not_change_results(ctx, b):
    """Launch shape and both step depths of the branch-free dictionary kernels
    are speed knobs only: packed windows (entries over 2^39) and, on the wide
    dictionary, windows spanning 2^53 or more, on a ragged column."""
    n = 300 * 1024 + 999
    for dct in (synth.dict_entries(min(1 << b, 4096), 23, b, 38), wide_dictionary(b)):
        m = len(dct)
        codes = synth.bounded(29, b, n, m)
        w = oracle.pack_rm(codes, b)
        col = api.encode_dict(codes, b, dct)
        for i, j in ((0, m - 1), (m // 3, m // 3 + max(1, m // 10)), (m // 2, m // 2)):
            lo, hi = int(dct[i]), int(dct[j]) + 1
            want = oracle.scan_dict(w, dct, n, b, lo, hi, zone_maps=True)
            for s in (strategy(DEC_RM_DIRECT, 0, 0), strategy(DEC_RM_DIRECT, 0, 1), strategy(DEC_RM_LDS, 0, 0)):
                for wg, per_cu, win, depth in ((64, 1, 1, 1), (128, 3, 5, 0), (256, 0, 64, 1), (192, 2, 0, 0),
                                               (0, 0, 0, 1)):
                    ctx.set_tune(ENC_DICT, b, s, wg, per_cu, win, depth)
                    got = ctx.run(col, lo, hi, s)
                    case = (b, m, s, wg, per_cu, win, depth, i, j)
                    assert (got["count"], got["sum"]) == (want.count, want.sum), case
                    if (s >> 3) & 1:
                        assert got["blocks_read"] == want.blocks_read, case
                ctx.set_tune(ENC_DICT, b, s, 0, 0, 0, 0)


def test_tune_file_round_trip_and_errors(ctx, tmp_path):
    """scan_tune_save / scan_tune_load: a saved file restores every entry; a
    file without entries or with a malformed or invalid entry is refused
    (SCAN_EINVAL) and installs nothing."""
    s = strategy(DEC_RM_DIRECT, 0, 0)
    ctx.set_tune(ENC_FOR, 7, s, 128, 2, 8, 1)
    good = str(tmp_path / "good.json")
    ctx.tune_save(good)
    ctx.set_tune(ENC_FOR, 7, s, 0, 0, 0)
    ctx.tune_load(good)
    assert ctx.get_tune(ENC_FOR, 7, s) == (128, 2, 8, 1)
    # a file written before the depth field existed loads with depth 0
    old = tmp_path / "old.json"
    old.write_text('{"format": "scan-autotune-1", "entries": [\n'
                   '  {"enc": 0, "b": 7, "strategy": %d, "wg_size": 64, "wgs_per_cu": 4, "window_blocks": 2}\n]}\n' % s)
    ctx.tune_load(str(old))
    assert ctx.get_tune(ENC_FOR, 7, s) == (64, 4, 2, 0)
    ctx.set_tune(ENC_FOR, 7, s, 0, 0, 0)
    before = ctx.get_tune(ENC_FOR, 7, s)
    cases = {
        "empty.json": '{"format": "scan-autotune-1", "entries": [\n]}\n',
        "garbled.json": '{"format": "scan-autotune-1", "entries": [\n'
                        '  {"enc": 0, "b": 7, "strategy": 1, "wg_size": 128, "wgs_per_cu": 2, "window_blocks": 8},\n'
                        '  {"enc": 0, "b": 9, "strategy": oops}\n]}\n',
        "invalid.json": '{"format": "scan-autotune-1", "entries": [\n'
                        '  {"enc": 0, "b": 7, "strategy": 1, "wg_size": 100, "wgs_per_cu": 2, "window_blocks": 8}\n]}\n',
        "bad_depth.json": '{"format": "scan-autotune-1", "entries": [\n'
                          '  {"enc": 0, "b": 7, "strategy": 1, "wg_size": 64, "wgs_per_cu": 2, "window_blocks": 8, '
                          '"depth": 2}\n]}\n',
    }
    for name, text in cases.items():
        path = tmp_path / name
        path.write_text(text)
        with pytest.raises(_lib.ScanError) as ei:
            ctx.tune_load(str(path))
        assert ei.value.status == _lib.SCAN_EINVAL, name
        assert ctx.get_tune(ENC_FOR, 7, s) == before, name
    with pytest.raises(_lib.ScanError):
        ctx.tune_load(str(tmp_path / "missing.json"))


def check_am(got, want, what):
    assert (got["count"], got["sum"], got["blocks_read"], got["blocks_total"]) == \
        (want.count, want.sum, want.blocks_read, want.blocks_total), (what, got, want)


def am_strategies(b, enc=ENC_FOR, li=False):
    if li:
        return [strategy(DEC_LI, sv, 1, 1) for sv in (0, 1)]
    decs = [DEC_RM_LDS, DEC_RM_DIRECT] + ([DEC_BYTES] if enc == ENC_FOR and b in (8, 16, 32) else [])
    return [strategy(d, sv, 1, 1) for d in decs for sv in (0, 1)]


@pytest.mark.parametrize("b", [1, 3, 8, 12, 16, 21, 31, 32])
def test_all_match_for(ctx, b):
    """Blocks entirely inside the predicate are counted from zone maps and
    block sums, not decoded: same COUNT and SUM, blocks_read as the oracle's
    all-match definition, in every decoder and predicate mode."""
    top = 1 << b
    for n in (1, 1024, 7 * 1024 + 99):
        raw = synth.width_values(synth.pcg32(91, b, n), b)
        srt = np.sort(raw)
        for v in (srt, srt[::-1].copy(), raw):
            w = oracle.pack_rm(v, b)
            col, coli = api.encode_for(v, b), api.encode_for(v, b, layout=LAYOUT_LI)
            preds = [(0, top), (int(srt[n // 3]), int(srt[2 * n // 3]) + 1), (int(srt[n // 2]), int(srt[n // 2]) + 1),
                     (top // 4, top // 2 + 1), (-3, 1 << 40), (5, 5)]
            for lo, hi in preds:
                want = oracle.scan_for(w, n, b, lo, hi, zone_maps=True, all_match=True)
                for s in am_strategies(b):
                    check_am(ctx.run(col, lo, hi, s), want, (b, n, lo, hi, _lib.strategy_name(s)))
                for s in am_strategies(b, li=True):
                    check_am(ctx.run(coli, lo, hi, s), want, (b, n, lo, hi, _lib.strategy_name(s)))
    # block references (per-block minimum) on sorted data
    n = 6 * 1024 + 5
    v = np.sort(synth.width_values(synth.pcg32(93, b, n), b)).astype(np.uint32)
    refs, codes = oracle.for_encode(v, b, policy=1)
    w = oracle.pack_rm(codes, b)
    col = api.encode_for(v, b, ref_policy=1)
    for lo, hi in [(int(v[1000]), int(v[5000]) + 1), (0, top)]:
        want = oracle.scan_for(w, n, b, lo, hi, refs=refs, zone_maps=True, all_match=True)
        for s in am_strategies(b):
            check_am(ctx.run(col, lo, hi, s), want, ("refs", b, lo, hi, _lib.strategy_name(s)))


@pytest.mark.parametrize("b", [1, 5, 16, 32])
def test_all_match_delta_and_dict(ctx, b):
    for n in (1, 2048, 5 * 1024 + 31):
        d = synth.width_values(synth.pcg32(94, b, n), b).astype(np.int64)
        v = np.cumsum(d) + 12345
        bases, codes = oracle.delta_encode(v, b)
        w = oracle.pack_rm(codes, b)
        col = api.encode_delta(v, b)
        for lo, hi in [(int(v[0]), int(v[-1]) + 1), (int(v[n // 4]), int(v[3 * n // 4]) + 1), (7, 7)]:
            want = oracle.scan_delta(w, bases, n, b, lo, hi, zone_maps=True, all_match=True)
            for s in am_strategies(b, ENC_DELTA):
                check_am(ctx.run(col, lo, hi, s), want, ("delta", b, n, lo, hi, _lib.strategy_name(s)))
        m = min(1 << b, 4096)
        dct = synth.dict_entries(m, 95, b, 38)
        cds = np.sort(synth.bounded(96, b, n, m)).astype(np.uint32)
        w = oracle.pack_rm(cds, b)
        col = api.encode_dict(cds, b, dct)
        for lo, hi in [(int(dct[0]), int(dct[-1]) + 1), (int(dct[m // 4]), int(dct[(3 * m) // 4])), (int(dct[0]) - 5, int(dct[0]))]:
            want = oracle.scan_dict(w, dct, n, b, lo, hi, zone_maps=True, all_match=True)
            for s in am_strategies(b, ENC_DICT):
                check_am(ctx.run(col, lo, hi, s), want, ("dict", b, n, lo, hi, _lib.strategy_name(s)))


def test_all_match_needs_block_sums_and_is_the_default(ctx):
    v = np.sort(synth.width_values(synth.pcg32(97, 10, 4096), 10))
    col = api.encode_for(v, 10)
    got = ctx.run(col, 100, 900, -1)
    assert got["strategy_used"] == strategy(DEC_RM_DIRECT, 0, 1, 1)
    bare = api.encode_for(v, 10, block_sums=False)
    assert ctx.run(bare, 100, 900, -1)["strategy_used"] == strategy(DEC_RM_DIRECT, 0, 1)
    with pytest.raises(_lib.ScanError):
        ctx.run(bare, 100, 900, strategy(DEC_RM_DIRECT, 0, 1, 1))
    with pytest.raises(_lib.ScanError):
        ctx.run(col, 100, 900, strategy(DEC_RM_DIRECT, 0, 0, 1))  # all-match without zone maps


def test_cache_flush_only_reads_its_buffer(ctx):
    """The eviction reads its scratch buffer (no dirty lines for the next
    kernel to write back); the contents stay as they were, and a scan
    launched after it is unchanged."""
    buf = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    want = buf.clone()
    for _ in range(3):
        ctx.cache_flush(buf, buf.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(buf, want)
    v = synth.width_values(synth.pcg32(11, 3, 5197), 12)
    col = api.encode_for(v, 12)
    r = ctx.run(col, 100, 900, strategy(DEC_RM_DIRECT, 0, 0))
    want = oracle.scan_for(oracle.pack_rm(v, 12), len(v), 12, 100, 900)
    assert (r["count"], r["sum"]) == (want.count, want.sum)
