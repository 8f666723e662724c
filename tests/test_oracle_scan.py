"""Pins of the oracle's scan: closed forms, brute force with Python integers,
zone-map invariants, and the dictionary's two equivalent predicate paths."""
import math

import numpy as np
import pytest

import oracle
import synth


def py_count_sum(values, lo, hi):
    """Brute force with Python integers: count and the exact sum, then mod 2^64 as int64."""
    sel = [int(v) for v in values if lo <= int(v) < hi] if lo < hi else []
    s = sum(sel)
    wrapped = ((s + (1 << 63)) % (1 << 64)) - (1 << 63)
    return len(sel), wrapped, s


def ap_closed_form(a, d, n, lo, hi):
    """v_i = a + d i: the matching i form [ceil((lo-a)/d), ceil((hi-a)/d)) & [0, n)."""
    if lo >= hi:
        return 0, 0
    if d == 0:
        return (n, n * a) if lo <= a < hi else (0, 0)
    i0 = max(0, -((a - lo) // d))     # ceil((lo - a) / d)
    i1 = min(n, -((a - hi) // d))     # ceil((hi - a) / d)
    k = max(0, i1 - i0)
    return k, k * (a + d * i0) + d * k * (k - 1) // 2


def sawtooth_closed_form(n, b, c):
    """v_i = i mod 2^b, predicate [0, c): q full periods and a remainder r."""
    period = 1 << b
    q, r = divmod(n, period)
    m = min(r, c)
    return q * c + m, q * c * (c - 1) // 2 + m * (m - 1) // 2


def zm_blocks_read(values, lo, hi):
    """Blocks whose [min, max] meets [lo, hi), from numpy min/max per block."""
    if lo >= hi or len(values) == 0:
        return 0
    nb = (len(values) + 1023) // 1024
    cnt = 0
    for k in range(nb):
        blk = values[k * 1024:(k + 1) * 1024]
        if not (int(blk.max()) < lo or int(blk.min()) >= hi):
            cnt += 1
    return cnt


@pytest.mark.parametrize("b", [1, 2, 3, 5, 8, 11, 16, 17, 24, 31, 32])
def test_arithmetic_progression_closed_form(b):
    n = 3 * 1024 + 333
    top = (1 << b) - 1
    for d in (0, 1, 3):
        a = 0 if d else top // 2
        if a + d * (n - 1) > top:
            d = top // (n - 1) if n > 1 else 0
        v = (a + d * np.arange(n, dtype=np.int64)).astype(np.uint32)
        w = oracle.pack_rm(v, b)
        for lo, hi in ((0, 1 << b), (a + d * 10, a + d * 500 + 1), (1, 1), (top, top + 1), (-5, 2)):
            want = ap_closed_form(a, d, n, lo, hi)
            for layout in (0, 1):
                pw = w if layout == 0 else oracle.pack_li(v, b)
                r = oracle.scan_for(pw, n, b, lo, hi, layout=layout)
                assert (r.count, r.sum) == want, (b, d, lo, hi, layout)


@pytest.mark.parametrize("b", [1, 2, 4, 7, 10])
def test_sawtooth_closed_form(b):
    n = 5 * 1024 + 17
    v = (np.arange(n) % (1 << b)).astype(np.uint32)
    w = oracle.pack_rm(v, b)
    for c in sorted({1, (1 << b) // 3 + 1, 1 << b}):
        r = oracle.scan_for(w, n, b, 0, c)
        assert (r.count, r.sum) == sawtooth_closed_form(n, b, c)


def test_brute_force_all_widths(rng):
    for b in range(1, 33):
        for n in (1, 700, 2100):
            v = rng.integers(0, 1 << b, size=n, dtype=np.uint64).astype(np.uint32)
            w = oracle.pack_rm(v, b)
            x = int(v[n // 2])
            preds = [(0, 1 << b), (x, x + 1), (5, 5), (9, 3), (-10, 0)]
            for _ in range(4):
                lo, hi = sorted(int(t) for t in rng.integers(-3, (1 << b) + 3, size=2))
                preds.append((lo, hi))
            for lo, hi in preds:
                cnt, s, _ = py_count_sum(v, lo, hi)
                for zm in (False, True):
                    r = oracle.scan_for(w, n, b, lo, hi, zone_maps=zm)
                    assert (r.count, r.sum) == (cnt, s), (b, n, lo, hi, zm)
                    if zm:
                        assert r.blocks_read == zm_blocks_read(v, lo, hi)
                    else:
                        assert r.blocks_read == (oracle.nblocks(n) if lo < hi else 0)


def test_reference_policy_matches_raw(rng):
    v = (rng.integers(0, 1 << 12, size=7000) + 50_000 * np.repeat(np.arange(7), 1024)[:7000]).astype(np.uint32)
    refs, codes = oracle.for_encode(v, 12, policy=1)
    w = oracle.pack_rm(codes, 12)
    for lo, hi in ((0, 1 << 32), (100_000, 210_000), (50_500, 50_501)):
        r = oracle.scan_for(w, len(v), 12, lo, hi, refs=refs, zone_maps=True)
        cnt, s, _ = py_count_sum(v, lo, hi)
        assert (r.count, r.sum) == (cnt, s)
        assert r.blocks_read == zm_blocks_read(v, lo, hi)


def test_count_sum_on_raw_values(rng):
    v = rng.integers(0, 1 << 32, size=10_000, dtype=np.uint64).astype(np.uint32)
    for lo, hi in ((0, 1 << 32), (1 << 31, 3 << 30)):
        r = oracle.count_sum(v, lo, hi)
        cnt, s, _ = py_count_sum(v, lo, hi)
        assert (r.count, r.sum) == (cnt, s)


def test_sum_wraps_mod_2_64():
    v = np.array([(1 << 62) + 5] * 5 + [-(1 << 62)], dtype=np.int64)
    r = oracle.count_sum(v, -(1 << 63), (1 << 63) - 1)
    cnt, s, exact = py_count_sum(v, -(1 << 63), (1 << 63) - 1)
    assert (r.count, r.sum) == (cnt, s) and r.sum_overflow and exact != s


def test_sorted_column_zone_maps_closed_form():
    """Sorted v_r = r >> 14: each value fills 16 whole blocks, so a predicate
    [lo, hi) reads exactly 16 (hi - lo) blocks and COUNT/SUM have closed forms."""
    n_distinct, rep = 64, 1 << 14
    n = n_distinct * rep
    v = (np.arange(n) >> 14).astype(np.uint32)
    w = oracle.pack_rm(v, 16)
    for lo, hi in ((0, 1), (5, 9), (0, 64), (63, 64), (10, 11)):
        r = oracle.scan_for(w, n, 16, lo, hi, zone_maps=True)
        assert r.count == (hi - lo) * rep
        assert r.sum == rep * (hi - lo) * (lo + hi - 1) // 2
        assert r.blocks_read == 16 * (hi - lo)
        off = oracle.scan_for(w, n, 16, lo, hi, zone_maps=False)
        assert (off.count, off.sum) == (r.count, r.sum) and off.blocks_read == n // 1024


def test_clustering_levels_are_one_multiset():
    """Every clustering level permutes the same multiset, so COUNT and SUM agree."""
    n, nd = 1 << 18, 1 << 4  # 2^14 copies of each value: 16 whole blocks when sorted
    cols = {s: synth.config3_column(n, nd, s).numpy().astype(np.uint32) for s in (0, 16, 1024, "random")}
    for lo, hi in ((0, 1), (7, 10), (0, 16)):
        res = {s: oracle.scan_for(oracle.pack_rm(c, 16), n, 16, lo, hi, zone_maps=True)
               for s, c in cols.items()}
        assert len({(r.count, r.sum) for r in res.values()}) == 1
        assert res[0].blocks_read == 16 * (hi - lo)
        assert res["random"].blocks_read == n // 1024


def test_random_data_skip_statistic():
    """i.i.d. uniform values on [0, V): a block of L values is skipped with
    probability (lo/V)^L + ((V-hi)/V)^L.  Checked loosely (binomial bounds)."""
    b, n = 16, 1024 * 2000
    V = 1 << b
    v = synth.width_values(synth.pcg32(99, 0, n), b)
    w = oracle.pack_rm(v, b)
    nb = n // 1024
    for width in (2, 7, 40):
        lo, hi = 1000, 1000 + width
        p_skip = (lo / V) ** 1024 + ((V - hi) / V) ** 1024
        r = oracle.scan_for(w, n, b, lo, hi, zone_maps=True)
        expect = nb * (1 - p_skip)
        sd = math.sqrt(nb * p_skip * (1 - p_skip)) + 1
        assert abs(r.blocks_read - expect) < 6 * sd, (width, r.blocks_read, expect)


def test_delta_scan_constant_delta_is_progression():
    b, n, a, d = 5, 4 * 1024 + 9, 1 << 40, 3
    v = a + d * np.arange(n, dtype=np.int64)
    bases, codes = oracle.delta_encode(v, b)
    w = oracle.pack_rm(codes, b)
    for lo, hi in ((a, a + 1), (a + 30, a + 3000), (0, 1 << 62), (a + 7, a + 8)):
        r = oracle.scan_delta(w, bases, n, b, lo, hi)
        assert (r.count, r.sum) == ap_closed_form(a, d, n, lo, hi)


def test_delta_scan_matches_brute_force(rng):
    for b in (1, 4, 9, 17, 24, 32):
        n = 3000
        d = rng.integers(0, 1 << b, size=n, dtype=np.uint64).astype(np.int64)
        d[0] = int(rng.integers(0, 1 << 32))
        v = np.cumsum(d)
        bases, codes = oracle.delta_encode(v, b)
        w = oracle.pack_rm(codes, b)
        for p, q in ((0, n - 1), (100, 1500), (2999, 2999)):
            lo, hi = int(v[p]), int(v[q]) + 1
            for zm in (False, True):
                r = oracle.scan_delta(w, bases, n, b, lo, hi, zone_maps=zm)
                cnt, s, _ = py_count_sum(v, lo, hi)
                assert (r.count, r.sum) == (cnt, s)
                if zm:
                    assert r.blocks_read == zm_blocks_read(v, lo, hi)


def test_dictionary_value_range_equals_code_range(rng):
    """Path A (value predicate on decoded values, inside the oracle) equals path B
    (code predicate [lower_bound(D, lo), lower_bound(D, hi)) on the codes)."""
    for b, m in ((3, 8), (10, 1000), (12, 4096), (20, 4096)):
        dct = np.cumsum(rng.integers(1, 1 << 20, size=m)).astype(np.int64) - (1 << 28)
        codes = rng.integers(0, m, size=5000).astype(np.uint32)
        w = oracle.pack_rm(codes, b)
        for _ in range(6):
            i, j = sorted(int(t) for t in rng.integers(0, m, size=2))
            lo = int(dct[i]) - int(rng.integers(0, 2))
            hi = int(dct[j]) + int(rng.integers(0, 2))
            clo, chi = np.searchsorted(dct, lo, "left"), np.searchsorted(dct, hi, "left")
            sel = (codes >= clo) & (codes < chi)
            want = (int(sel.sum()), int(sum(int(x) for x in dct[codes[sel]])))
            r = oracle.scan_dict(w, dct, len(codes), b, lo, hi, zone_maps=True)
            assert (r.count, r.sum) == want
            zb = sum(1 for k in range(5) if not (codes[k * 1024:(k + 1) * 1024].max() < clo
                                                 or codes[k * 1024:(k + 1) * 1024].min() >= chi))
            assert r.blocks_read == (zb if lo < hi else 0)


def test_query_matches_numpy(rng):
    n = 6000
    a = rng.integers(0, 256, size=n).astype(np.uint32)
    dct = np.cumsum(rng.integers(1, 99, size=64)).astype(np.int64) - 1000
    c = rng.integers(0, 64, size=n).astype(np.uint32)
    s = rng.integers(0, 1 << 20, size=n).astype(np.uint32)
    cols = [dict(enc=0, b=8, payload=oracle.pack_rm(a, 8)),
            dict(enc=2, b=6, payload=oracle.pack_rm(c, 6), dict=dct),
            dict(enc=0, b=20, payload=oracle.pack_rm(s, 20))]
    for filters in ([(0, 10, 100)], [(0, 0, 50), (1, int(dct[3]), int(dct[40]))],
                    [(1, -5000, 5000), (0, 7, 8), (2, 0, 1 << 19)]):
        mask = np.ones(n, dtype=bool)
        for col, lo, hi in filters:
            val = (a, dct[c], s)[col].astype(np.int64)
            mask &= (val >= lo) & (val < hi)
        for sc in (2, 1):
            val = (a, dct[c], s)[sc].astype(np.int64)
            r = oracle.query(cols, n, filters, sc)
            assert (r.count, r.sum) == (int(mask.sum()), int(sum(int(x) for x in val[mask])))


def _numpy_block_masks(v, lo, hi):
    """(survives, inside) per 1024-value block, from numpy min/max."""
    nb = (len(v) + 1023) // 1024
    mn = np.array([v[k * 1024:(k + 1) * 1024].min() for k in range(nb)], dtype=np.int64)
    mx = np.array([v[k * 1024:(k + 1) * 1024].max() for k in range(nb)], dtype=np.int64)
    survive = ~((mx < lo) | (mn >= hi))
    inside = (mn >= lo) & (mx < hi)
    return survive, inside


@pytest.mark.parametrize("n", [1, 1023, 1024, 5 * 1024 + 77])
def test_all_match_counts_only_blocks_not_entirely_inside(rng, n):
    """The all-match extension leaves COUNT and SUM alone; blocks_read drops
    the surviving blocks whose [min, max] lies inside [lo, hi)."""
    b = 12
    base = np.sort(rng.integers(0, 1 << b, size=n)).astype(np.uint32)  # clustered: many blocks inside
    for v in (base, rng.permutation(base)):
        w = oracle.pack_rm(v, b)
        for lo, hi in [(0, 1 << b), (100, 3000), (int(v[n // 2]), int(v[n // 2]) + 1), (5, 5), (-7, 1 << 40)]:
            zm = oracle.scan_for(w, n, b, lo, hi, zone_maps=True)
            am = oracle.scan_for(w, n, b, lo, hi, zone_maps=True, all_match=True)
            assert (am.count, am.sum) == (zm.count, zm.sum)
            if lo >= hi:
                assert am.blocks_read == 0
                continue
            survive, inside = _numpy_block_masks(v.astype(np.int64), lo, hi)
            assert zm.blocks_read == int(survive.sum())
            assert am.blocks_read == int((survive & ~inside).sum())
    # all-match without zone maps is ignored (the shortcut needs the zone maps)
    w = oracle.pack_rm(base, b)
    off = oracle.scan_for(w, n, b, 0, 1 << b, zone_maps=False, all_match=True)
    assert off.blocks_read == (n + 1023) // 1024


def test_all_match_on_the_sorted_column_reads_only_edge_blocks():
    """Sorted values v_r = r >> 4: a predicate whose edges fall inside blocks
    reads exactly those (at most two) edge blocks."""
    n = 1 << 16
    v = (np.arange(n) >> 4).astype(np.uint32)  # 64 distinct values per block
    w = oracle.pack_rm(v, 12)
    for lo, hi, edges in [(64, 128, 0), (70, 128, 1), (64, 1000, 1), (70, 1000, 2), (70, 75, 1)]:
        r = oracle.scan_for(w, n, 12, lo, hi, zone_maps=True, all_match=True)
        assert r.blocks_read == edges, (lo, hi, r)
        assert r.count == 16 * (hi - lo)
        assert r.sum == 16 * (hi - lo) * (lo + hi - 1) // 2


def test_all_match_delta_and_dictionary(rng):
    n = 3 * 1024 + 5
    d = rng.integers(0, 8, size=n).astype(np.int64)
    v = np.cumsum(d) + 1000
    bases, codes = oracle.delta_encode(v, 3)
    w = oracle.pack_rm(codes, 3)
    lo, hi = int(v[100]), int(v[2500])
    zm = oracle.scan_delta(w, bases, n, 3, lo, hi, zone_maps=True)
    am = oracle.scan_delta(w, bases, n, 3, lo, hi, zone_maps=True, all_match=True)
    survive, inside = _numpy_block_masks(v, lo, hi)
    assert (am.count, am.sum) == (zm.count, zm.sum)
    assert am.blocks_read == int((survive & ~inside).sum()) and int(inside.sum()) >= 1
    dct = np.arange(0, 4096 * 3, 3, dtype=np.int64) - 5000
    codes = np.sort(rng.integers(0, 4096, size=n)).astype(np.uint32)
    w = oracle.pack_rm(codes, 12)
    lo, hi = int(dct[500]), int(dct[3000])
    zm = oracle.scan_dict(w, dct, n, 12, lo, hi, zone_maps=True)
    am = oracle.scan_dict(w, dct, n, 12, lo, hi, zone_maps=True, all_match=True)
    survive, inside = _numpy_block_masks(dct[codes], lo, hi)
    assert (am.count, am.sum) == (zm.count, zm.sum)
    assert am.blocks_read == int((survive & ~inside).sum()) and int(inside.sum()) >= 1


@pytest.mark.parametrize("b", [1, 7, 16, 32])
def test_select_is_the_plain_position_list(rng, b):
    """Materializing select = numpy's nonzero on the raw values; refine and
    gather are the same definition applied to a position list."""
    for n in (0, 1, 1023, 1025, 4 * 1024 + 9):
        v = rng.integers(0, 1 << b, size=n, dtype=np.uint64).astype(np.uint32)
        w = oracle.pack_rm(v, b)
        wl = oracle.pack_li(v, b)
        for lo, hi in [(0, 1 << b), (5, 5), (1 << (b - 1), (1 << b) - 1), (-4, 3)]:
            want = np.nonzero((v.astype(np.int64) >= lo) & (v.astype(np.int64) < hi))[0].astype(np.uint32)
            got = oracle.select(0, w, n, b, lo, hi)
            assert np.array_equal(got, want)
            assert np.array_equal(oracle.select(0, wl, n, b, lo, hi, layout=1), want)
            r = oracle.scan_for(w, n, b, lo, hi)
            assert r.count == len(got) and r.sum == int(v[got].astype(np.uint64).sum())
            assert np.array_equal(oracle.gather(0, w, b, got), v[got].astype(np.int64))
            lo2, hi2 = 0, (1 << b) // 3 + 1
            ref = oracle.refine(0, w, b, lo2, hi2, got)
            assert np.array_equal(ref, got[(v[got] >= lo2) & (v[got] < hi2)])
    # dictionary: values are entries
    m = min(1 << b, 4096)
    dct = np.sort(rng.choice(np.arange(-(1 << 36), 1 << 36, 1 << 20), size=m, replace=False)).astype(np.int64)
    codes = rng.integers(0, m, size=3000).astype(np.uint32)
    w = oracle.pack_rm(codes, b)
    lo, hi = int(dct[m // 4]), int(dct[(3 * m) // 4]) + 1
    want = np.nonzero((dct[codes] >= lo) & (dct[codes] < hi))[0].astype(np.uint32)
    assert np.array_equal(oracle.select(2, w, 3000, b, lo, hi, dct=dct), want)
    assert np.array_equal(oracle.gather(2, w, b, want, dct=dct), dct[codes[want]])


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 5 * 1024 + 77])
def test_zonemaps_are_per_block_min_max_of_valid_values(rng, n):
    """The oracle's zone maps (the paper's per-block min/max, "Method") against
    numpy's reductions over each 1024-value block, the last block holding only
    its n - 1024 k valid values: a partial block must not count its padding
    (a padded zero would lower the minimum, a padded extreme raise the
    maximum)."""
    L = 1024
    nb = (n + L - 1) // L
    # u32: values kept away from 0 so a counted padding slot would show
    v = rng.integers(1 << 20, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    mn, mx = oracle.zonemap_u32(v)
    assert mn.shape == (nb,) and mx.shape == (nb,)
    for k in range(nb):
        blk = v[k * L: min(n, (k + 1) * L)]
        assert int(mn[k]) == int(blk.min()) and int(mx[k]) == int(blk.max()), (n, k)
    # int64, including both extremes of the type
    w = rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    w[0] = np.iinfo(np.int64).min
    w[-1] = np.iinfo(np.int64).max
    if n > 2:
        w[n // 2] = -1
    mn, mx = oracle.zonemap_i64(w)
    for k in range(nb):
        blk = w[k * L: min(n, (k + 1) * L)]
        assert int(mn[k]) == int(blk.min()) and int(mx[k]) == int(blk.max()), (n, k)
    # an all-negative partial last block: padding read as 0 would become the maximum
    z = -rng.integers(1, 1 << 40, size=n, dtype=np.int64)
    mn, mx = oracle.zonemap_i64(z)
    assert int(mx[-1]) == int(z[(nb - 1) * L:].max()) < 0
