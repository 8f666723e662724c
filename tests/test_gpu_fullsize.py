"""GPU parity at the sizes and launch shapes the benchmark runs.

* Closed-form columns of N = 2^28 values (the bit-width sweep's length), every
  decoder x predicate mode, zone maps on and off, the library's default launch
  shapes (a wavefront walks many windows, each of many pipelined steps).  The
  payload is packed on the GPU by a third packer written here from the format
  text (neither the library's encoder nor the oracle's), and the expected COUNT
  and SUM are closed forms in Python integers:
    sawtooth  v_i = i mod 2^b, n = q 2^b + r: every period holds 0 .. 2^b - 1
              once, the last r values 0 .. r - 1, so COUNT = q |[lo,hi) & [0,2^b)|
              + |[lo,hi) & [0,r)| and SUM likewise with S(a, c) = (c - a)(a + c - 1)/2;
    progression v_i = a + d i: the matches are i in [ceil((lo-a)/d), ceil((hi-a)/d)) & [0, n).
  With zone maps, blocks_read is the count of blocks whose (closed-form) value
  range meets the predicate.
* Random columns of 2^24 values that the oracle packs itself: the GPU scans the
  oracle's payload, and every result equals the oracle's scan of it, with the
  default launch shape and with one that makes each wavefront walk 16 windows.
* A 2^24-row materializing select compared element by element with the oracle.
Tolerance 0 (integers)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2606_22423_amd import api  # noqa: E402
from paper_2606_22423_amd._lib import (DEC_BYTES, DEC_LI, DEC_RM_DIRECT, DEC_RM_LDS, ENC_DICT, ENC_FOR,  # noqa: E402
                                       LAYOUT_LI, LAYOUT_RM, strategy)

N28 = 1 << 28
L = 1024


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


# ------------------------------------------------------------ GPU packer
def pack_gpu(v, b: int, layout: int):
    """Payload words (int32 tensor) of the u32 values v (int64 tensor on the
    GPU): 1024-value blocks of 32 b words; row-major: value j of a block at
    block bits [j b, j b + b); lane-interleaved: value j to lane j mod 32, slot
    j div 32, lane bit t at block word 32 (t div 32) + lane; bits LSB first.
    Fields never overlap, so adding the shifted pieces sets them."""
    n = v.numel()
    nb = (n + L - 1) // L
    words = torch.zeros(nb * 32 * b, dtype=torch.int64, device=v.device)
    i = torch.arange(n, dtype=torch.int64, device=v.device)
    k, j = i >> 10, i & (L - 1)
    if layout == LAYOUT_RM:
        t = j * b
        w = k * (32 * b) + (t >> 5)
        step = 1
    else:
        lane, slot = j & 31, j >> 5
        t = slot * b
        w = k * (32 * b) + (t >> 5) * 32 + lane
        step = 32
    del i, j
    sh = t & 31
    del t
    words.index_add_(0, w, (v << sh) & 0xFFFFFFFF)
    spill = (sh + b) > 32
    if bool(spill.any()):
        words.index_add_(0, w[spill] + step, v[spill] >> (32 - sh[spill]))
    del w, sh, spill
    return (words - ((words >= (1 << 31)).to(torch.int64) << 32)).to(torch.int32)


def sawtooth(n: int, b: int, device="cuda"):
    return torch.arange(n, dtype=torch.int64, device=device) & ((1 << b) - 1)


def s_range(a: int, c: int) -> int:
    """sum of x for a <= x < c (0 if empty)."""
    return 0 if c <= a else (c - a) * (a + c - 1) // 2


def sawtooth_closed(n: int, b: int, lo: int, hi: int):
    p = 1 << b
    q, r = divmod(n, p)
    a1, c1 = max(lo, 0), min(hi, p)
    a2, c2 = max(lo, 0), min(hi, r)
    cnt = q * max(0, c1 - a1) + max(0, c2 - a2)
    tot = q * s_range(a1, c1) + s_range(a2, c2)
    return cnt, tot


def progression_closed(n: int, a: int, d: int, lo: int, hi: int):
    def first_at_least(x):  # smallest i with a + d i >= x
        return max(0, -((a - x) // d))
    i0, i1 = min(first_at_least(lo), n), min(first_at_least(hi), n)
    k = max(0, i1 - i0)
    return k, k * (a + d * i0) + d * k * (k - 1) // 2


def to_i64(x: int) -> int:
    x %= 1 << 64
    return x - (1 << 64) if x >= 1 << 63 else x


def zone_maps(v):
    blk = v.view(-1, L) if v.numel() % L == 0 else None
    assert blk is not None
    return blk.amin(1), blk.amax(1)


def as_u32(t):
    return (t - ((t >= (1 << 31)).to(torch.int64) << 32)).to(torch.int32)


def make_column(v, b, layout):
    zmin, zmax = zone_maps(v)
    return api.Column(ENC_FOR, b, v.numel(), layout, pack_gpu(v, b, layout), zmin=as_u32(zmin), zmax=as_u32(zmax)), \
        zmin, zmax


def blocks_meeting(zmin, zmax, lo, hi):
    if lo >= hi:
        return 0
    return int(((zmax >= lo) & (zmin < hi)).sum().item())


def strategies_for(b, layout):
    if layout == LAYOUT_LI:
        return [strategy(DEC_LI, sv, zm) for sv in (0, 1) for zm in (0, 1)]
    decs = [DEC_RM_LDS, DEC_RM_DIRECT] + ([DEC_BYTES] if b in (8, 16, 32) else [])
    return [strategy(d, sv, zm) for d in decs for sv in (0, 1) for zm in (0, 1)]


def predicates(b):
    p = 1 << b
    out = [(0, max(1, round(0.1 * p))), (p // 3, p // 3 + max(1, p // 7)), (0, p), (p - 1, p + 5)]
    if b >= 2:
        out.append((1, 2))
    return out


@pytest.mark.parametrize("b", [1, 2, 3, 5, 6, 7, 8, 9, 11, 12, 15, 16, 23, 24, 31, 32])
def test_sawtooth_full_size_every_decoder(ctx, b):
    v = sawtooth(N28, b)
    for layout in (LAYOUT_RM, LAYOUT_LI):
        col, zmin, zmax = make_column(v, b, layout)
        for lo, hi in predicates(b):
            cnt, tot = sawtooth_closed(N28, b, lo, hi)
            want_blocks = blocks_meeting(zmin, zmax, lo, hi)
            for s in strategies_for(b, layout):
                say("sawtooth n=2^28 b=%d layout=%d strategy=%d pred=[%d,%d)" % (b, layout, s, lo, hi))
                got = ctx.run(col, lo, hi, s)
                assert (got["count"], got["sum"]) == (cnt, to_i64(tot)), (b, layout, s, lo, hi, got, cnt, tot)
                want_read = want_blocks if (s >> 3) & 1 else N28 // L
                assert got["blocks_read"] == want_read and got["blocks_total"] == N28 // L, (b, s, lo, hi, got)
        del col
    del v
    torch.cuda.empty_cache()


@pytest.mark.parametrize("b,a,d", [(30, 11, 3), (31, 5, 7), (32, 123456789, 13)])
def test_progression_full_size(ctx, b, a, d):
    assert a + d * (N28 - 1) < (1 << b)
    v = a + d * torch.arange(N28, dtype=torch.int64, device="cuda")
    for layout in (LAYOUT_RM, LAYOUT_LI):
        col, zmin, zmax = make_column(v, b, layout)
        top = a + d * N28
        for lo, hi in ((0, a + d * 1000), (a + d * (N28 // 3) + 1, a + d * (N28 // 2)), (0, 1 << b),
                       (top - d * 5000 - 1, 1 << 40), (a + 7, a + 8)):
            cnt, tot = progression_closed(N28, a, d, lo, hi)
            want_blocks = blocks_meeting(zmin, zmax, lo, hi)
            for s in strategies_for(b, layout):
                say("progression n=2^28 b=%d layout=%d strategy=%d pred=[%d,%d)" % (b, layout, s, lo, hi))
                got = ctx.run(col, lo, hi, s)
                assert (got["count"], got["sum"]) == (cnt, to_i64(tot)), (b, layout, s, lo, hi, got, cnt, tot)
                if (s >> 3) & 1:
                    assert got["blocks_read"] == want_blocks, (b, s, lo, hi, got, want_blocks)
        del col
    del v
    torch.cuda.empty_cache()


# ------------------------------------------------ oracle-packed 2^24 columns
N24 = 1 << 24


@pytest.mark.parametrize("b", [1, 3, 4, 5, 6, 7, 8, 10, 12, 16, 17, 24, 27, 32])
def test_oracle_packed_random_columns(ctx, b):
    raw = synth.width_values(synth.pcg32(811, b, N24), b)
    for layout, pack in ((LAYOUT_RM, oracle.pack_rm), (LAYOUT_LI, oracle.pack_li)):
        words = pack(raw, b)
        zmin, zmax = oracle.zonemap_u32(raw)
        col = api.Column(ENC_FOR, b, N24, layout, torch.from_numpy(words.view(np.int32)).cuda(),
                         zmin=torch.from_numpy(zmin.view(np.int32)).cuda(),
                         zmax=torch.from_numpy(zmax.view(np.int32)).cuda())
        p = 1 << b
        for lo, hi in ((0, max(1, p // 10)), (p // 4, p // 4 + max(1, p // 3)), (int(raw[77]), int(raw[77]) + 1)):
            want = oracle.scan_for(words, N24, b, lo, hi, layout=layout, zone_maps=True)
            for s in strategies_for(b, layout):
                for shape in ((0, 0, 0, 0), (64, 1, 4, 0), (0, 0, 0, 1)):
                    if any(shape):
                        # (64, 1, 4): 256 wavefronts of 4-block windows, every wavefront walks
                        # 16 windows; (0, 0, 0, 1): the alternative step depth
                        ctx.set_tune(ENC_FOR, b, s, *shape)
                    say("oracle-packed n=2^24 b=%d layout=%d strategy=%d shape=%s pred=[%d,%d)" %
                        (b, layout, s, shape, lo, hi))
                    got = ctx.run(col, lo, hi, s)
                    ctx.set_tune(ENC_FOR, b, s, 0, 0, 0)
                    assert (got["count"], got["sum"]) == (want.count, want.sum), (b, layout, s, shape, lo, hi)
                    if (s >> 3) & 1:
                        assert got["blocks_read"] == want.blocks_read, (b, layout, s, shape, lo, hi)
        del col


@pytest.mark.parametrize("b", [4, 8, 12])
def test_oracle_packed_dictionary_columns(ctx, b):
    """2^24 codes packed by the oracle over 2^b sorted entries spanning 2^39
    (the dictionary workload's shape), windows of 10 % and of one code, every
    row-major strategy at the default launch shape (the one the bench starts
    from) and at both step depths of the branch-free direct kernel."""
    m = 1 << b
    codes = synth.bounded(613, b, N24, m)
    dct = synth.dict_entries(m, 614, b, 38)
    words = oracle.pack_rm(codes, b)
    zmin, zmax = oracle.zonemap_u32(codes)
    col = api.Column(ENC_DICT, b, N24, LAYOUT_RM, torch.from_numpy(words.view(np.int32)).cuda(),
                     zmin=torch.from_numpy(zmin.view(np.int32)).cuda(),
                     zmax=torch.from_numpy(zmax.view(np.int32)).cuda(),
                     dct=torch.from_numpy(dct).cuda())
    cw = max(1, round(0.1 * m))
    c0 = (m - cw) // 2
    for i, j in ((c0, c0 + cw), (int(codes[77]), int(codes[77]) + 1)):
        lo, hi = int(dct[i]), int(dct[j]) if j < m else int(dct[m - 1]) + 1
        want = oracle.scan_dict(words, dct, N24, b, lo, hi, zone_maps=True)
        for s in [strategy(d, sv, zm) for d in (DEC_RM_DIRECT, DEC_RM_LDS) for sv in (0, 1) for zm in (0, 1)]:
            for depth in (0, 1):
                if depth:
                    ctx.set_tune(ENC_DICT, b, s, 0, 0, 0, 1)
                say("dictionary n=2^24 b=%d strategy=%d depth=%d pred=[%d,%d)" % (b, s, depth, lo, hi))
                got = ctx.run(col, lo, hi, s)
                ctx.set_tune(ENC_DICT, b, s, 0, 0, 0, 0)
                assert (got["count"], got["sum"]) == (want.count, want.sum), (b, s, depth, i, j)
                if (s >> 3) & 1:
                    assert got["blocks_read"] == want.blocks_read, (b, s, depth, i, j)
    del col


@pytest.mark.parametrize("b", [8, 21])
def test_select_2p24_matches_oracle(ctx, b):
    raw = synth.width_values(synth.pcg32(905, b, N24), b)
    words = oracle.pack_rm(raw, b)
    col = api.encode_for(raw, b)
    p = 1 << b
    for lo, hi in ((0, max(1, p // 1000)), (p // 3, p // 3 + p // 10)):
        want = oracle.select(0, words, N24, b, lo, hi)
        for zm in (False, True):
            say("select n=2^24 b=%d pred=[%d,%d) zone maps %s" % (b, lo, hi, zm))
            got = ctx.select(col, lo, hi, zone_maps=zm).cpu().numpy().view(np.uint32)
            assert got.shape == want.shape and np.array_equal(got, want), (b, lo, hi, zm, len(got), len(want))
