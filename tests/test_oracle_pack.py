"""Pins of the oracle's packing and decoding against definitions it does not share.

The independent decoder here reads a block as ONE Python integer built from the
payload's little-endian bytes and slices bits from it; the oracle's C code sets
and extracts bits with word arithmetic.  A wrong bit order, word index or shift
in either shows up as a mismatch.
"""
import numpy as np
import pytest

import oracle

EDGE_N = (0, 1, 31, 32, 33, 1023, 1024, 1025, 3 * 1024 + 7)


def bigint_decode_rm(words, n, b):
    mask = (1 << b) - 1
    out = []
    for k in range((n + 1023) // 1024):
        blk = np.asarray(words[k * 32 * b:(k + 1) * 32 * b], dtype="<u4").tobytes()
        big = int.from_bytes(blk, "little")
        for j in range(min(1024, n - 1024 * k)):
            out.append((big >> (j * b)) & mask)
    return np.array(out, dtype=np.uint64)


def bigint_decode_li(words, n, b):
    mask = (1 << b) - 1
    out = np.zeros(n, dtype=np.uint64)
    for k in range((n + 1023) // 1024):
        blk = np.asarray(words[k * 32 * b:(k + 1) * 32 * b], dtype=np.uint64)
        for lane in range(32):
            big = 0
            for r in range(b):
                big |= int(blk[32 * r + lane]) << (32 * r)
            for slot in range(32):
                i = 1024 * k + 32 * slot + lane
                if i < n:
                    out[i] = (big >> (slot * b)) & mask
    return out


def codes_for(rng, n, b):
    hi = 1 << b
    c = rng.integers(0, hi, size=n, dtype=np.uint64)
    if n >= 4:  # extremal values
        c[0], c[1], c[-1], c[-2] = 0, hi - 1, hi - 1, 0
    return c.astype(np.uint32)


@pytest.mark.parametrize("b", range(1, 33))
def test_round_trip_both_layouts(rng, b):
    for n in EDGE_N:
        c = codes_for(rng, n, b)
        for layout, pack in ((0, oracle.pack_rm), (1, oracle.pack_li)):
            w = pack(c, b)
            assert len(w) == oracle.nblocks(n) * 32 * b
            assert np.array_equal(oracle.unpack(w, n, b, layout), c), (b, n, layout)


@pytest.mark.parametrize("b", range(1, 33))
def test_against_bigint_decoder(rng, b):
    n = 2 * 1024 + 77
    c = codes_for(rng, n, b)
    assert np.array_equal(bigint_decode_rm(oracle.pack_rm(c, b), n, b), c.astype(np.uint64))
    if b in (1, 3, 5, 7, 8, 13, 16, 21, 31, 32):  # the lane decoder is slow in Python
        assert np.array_equal(bigint_decode_li(oracle.pack_li(c, b), n, b), c.astype(np.uint64))


@pytest.mark.parametrize("b,dt", [(8, np.uint8), (16, np.uint16), (32, np.uint32)])
def test_byte_aligned_widths_are_plain_arrays(rng, b, dt):
    """Byte-aligned widths coincide with plain little-endian integer arrays."""
    n = 5 * 1024 + 300
    c = codes_for(rng, n, b)
    w = oracle.pack_rm(c, b)
    raw = c.astype(np.dtype(dt).newbyteorder("<")).tobytes()
    padded = raw + b"\0" * (len(w) * 4 - len(raw))
    assert w.astype("<u4").tobytes() == padded


def test_lane_layout_special_widths(rng):
    n = 2048
    c = codes_for(rng, n, 32)
    # b = 32: lane l, slot t sits in word 32 t + l, i.e. word j holds value j
    assert np.array_equal(oracle.pack_li(c, 32), c)
    c16 = codes_for(rng, n, 16)
    w = oracle.pack_li(c16, 16).reshape(2, 16, 32)  # block, lane-word r, lane
    for k in range(2):
        for r in range(16):
            lanes = np.arange(32)
            lo = c16[1024 * k + 64 * r + lanes].astype(np.uint64)
            hi = c16[1024 * k + 64 * r + 32 + lanes].astype(np.uint64)
            assert np.array_equal(w[k, r].astype(np.uint64), lo | (hi << 16))


def test_layouts_decode_same_values(rng):
    for b in (1, 2, 7, 12, 19, 30):
        n = 4096 + 5
        c = codes_for(rng, n, b)
        assert np.array_equal(oracle.unpack(oracle.pack_rm(c, b), n, b, 0),
                              oracle.unpack(oracle.pack_li(c, b), n, b, 1))


def test_tail_slots_are_zero(rng):
    b, n = 11, 1024 + 10
    w = oracle.pack_rm(codes_for(rng, n, b), b)
    tail_block = w[32 * b:]
    start_bit = 10 * b
    big = int.from_bytes(tail_block.astype("<u4").tobytes(), "little")
    assert big >> start_bit == 0


def test_pack_rejects_wide_codes():
    with pytest.raises(ValueError):
        oracle.pack_rm(np.array([4], dtype=np.uint32), 2)
    with pytest.raises(ValueError):
        oracle.pack_li(np.array([1 << 20], dtype=np.uint32), 20)


def test_for_encode_policies(rng):
    v = rng.integers(1000, 1000 + 255, size=3000, dtype=np.uint32)
    refs, codes = oracle.for_encode(v, 8, policy=1)
    blocks = [v[k * 1024:(k + 1) * 1024] for k in range(3)]
    assert list(refs) == [int(x.min()) for x in blocks]
    assert np.array_equal(codes.astype(np.int64) + np.repeat(refs, 1024)[:3000], v.astype(np.int64))
    with pytest.raises(ValueError):
        oracle.for_encode(v, 8, policy=0)  # 1000 + x does not fit 8 bits without a reference


def test_delta_round_trip_and_rejections(rng):
    d = rng.integers(0, 1 << 9, size=4000).astype(np.int64)
    v = np.cumsum(d) + 123456789
    bases, codes = oracle.delta_encode(v, 9)
    assert list(bases) == [int(v[k * 1024]) for k in range(4)]
    assert np.all(codes[::1024] == 0)
    assert np.array_equal(oracle.delta_decode(codes, bases), v)
    with pytest.raises(ValueError):
        oracle.delta_encode(v, 8 if d.max() >= 256 else 1)
    with pytest.raises(ValueError):
        oracle.delta_encode(v[::-1].copy(), 9)


def test_dict_encode(rng):
    dct = np.cumsum(rng.integers(1, 1000, size=300)).astype(np.int64) - 5000
    codes = rng.integers(0, 300, size=2000).astype(np.uint32)
    assert np.array_equal(oracle.dict_encode(dct[codes], dct), codes)
    with pytest.raises(ValueError):
        oracle.dict_encode(np.array([dct[0] - 1]), dct)


def test_rle_round_trip_and_block_boundaries(rng):
    """Run-length format: runs never cross a 1024-value block, the lengths of
    a block sum to its value count, and decoding gives the values back."""
    for n in (0, 1, 1023, 1024, 1025, 5000):
        for v in (np.repeat(rng.integers(0, 50, size=n // 7 + 1), 7)[:n].astype(np.uint32),
                  rng.integers(0, 3, size=n).astype(np.uint32), np.zeros(n, dtype=np.uint32)):
            rv, rl, br = oracle.rle_encode(v)
            nb = (n + 1023) // 1024
            assert len(br) == nb + 1 and br[0] == 0 and br[-1] == len(rv)
            for k in range(nb):
                lens = rl[br[k]:br[k + 1]].astype(np.int64)
                assert lens.sum() == min(1024, n - 1024 * k) and lens.min() >= 1
                vals = rv[br[k]:br[k + 1]]
                assert np.all(vals[1:] != vals[:-1])  # maximal runs inside a block
            assert np.array_equal(oracle.rle_decode(rv, rl, br), v)
    # a constant column has exactly one run per block
    rv, rl, br = oracle.rle_encode(np.full(4096 + 3, 9, dtype=np.uint32))
    assert len(rv) == 5 and list(rl) == [1024] * 4 + [3]
