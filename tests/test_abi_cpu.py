"""CPU checks of the C ABI library: it loads, exports what include/scan.h
declares, and its host encoders produce byte-for-byte the oracle's packing
(two independent implementations of one format text)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2606_22423_amd import _lib, api


def test_library_exports_every_declared_function():
    lib = _lib.load()
    declared = _lib.header_functions()
    assert "scan_run" in declared and "scan_create" in declared
    missing = [f for f in declared if not hasattr(lib, f)]
    assert not missing, missing
    undeclared = [f for f in _lib.SIGNATURES if f not in declared]
    assert not undeclared, undeclared


def test_null_context_is_rejected_without_a_gpu():
    lib = _lib.load()
    r = _lib.ScanResult()
    assert lib.scan_run(None, None, 0, 8, None, 3, -1, ctypes.byref(r)) == _lib.SCAN_EINVAL
    assert lib.scan_sync(None) == _lib.SCAN_EINVAL
    assert lib.scan_last_error(None) == b"null context"


@pytest.mark.parametrize("b", range(1, 33))
def test_for_encoder_matches_oracle_packing(rng, b):
    for n in (1, 1023, 1025, 3 * 1024 + 5):
        v = rng.integers(0, 1 << b, size=n, dtype=np.uint64).astype(np.uint32)
        for layout, pack in ((0, oracle.pack_rm), (1, oracle.pack_li)):
            payload, refs, zmin, zmax = api.host_encode_for(v, b, layout)
            assert refs is None
            assert np.array_equal(payload, pack(v, b)), (b, n, layout)
            omin, omax = oracle.zonemap_u32(v)
            assert np.array_equal(zmin, omin) and np.array_equal(zmax, omax)


def test_for_encoder_reference_policy(rng):
    v = (rng.integers(0, 1 << 10, size=5000) + 7_000_000).astype(np.uint32)
    payload, refs, zmin, zmax = api.host_encode_for(v, 10, ref_policy=1)
    orefs, codes = oracle.for_encode(v, 10, policy=1)
    assert np.array_equal(refs, orefs)
    assert np.array_equal(payload, oracle.pack_rm(codes, 10))
    with pytest.raises(_lib.ScanError):
        api.host_encode_for(v, 10, ref_policy=0)


@pytest.mark.parametrize("b", [1, 3, 8, 13, 22, 23, 31, 32])
def test_delta_encoder_matches_oracle(rng, b):
    n = 4 * 1024 + 99
    d = rng.integers(0, 1 << b, size=n, dtype=np.uint64).astype(np.int64)
    v = np.cumsum(d) - (1 << 40)
    payload, bases, zmin, zmax = api.host_encode_delta(v, b)
    obases, codes = oracle.delta_encode(v, b)
    assert np.array_equal(bases, obases)
    assert np.array_equal(payload, oracle.pack_rm(codes, b))
    omin, omax = oracle.zonemap_i64(v)
    assert np.array_equal(zmin, omin) and np.array_equal(zmax, omax)
    with pytest.raises(_lib.ScanError):
        api.host_encode_delta(v[::-1].copy(), b)


@pytest.mark.parametrize("b,m", [(1, 2), (5, 32), (12, 4096), (20, 4096)])
def test_dict_encoder_matches_oracle(rng, b, m):
    codes = rng.integers(0, m, size=3000).astype(np.uint32)
    payload, zmin, zmax = api.host_encode_dict(codes, b, m)
    assert np.array_equal(payload, oracle.pack_rm(codes, b))
    omin, omax = oracle.zonemap_u32(codes)
    assert np.array_equal(zmin, omin) and np.array_equal(zmax, omax)
    with pytest.raises(_lib.ScanError):
        api.host_encode_dict(codes, b, int(codes.max()))  # a code equal to dict_len is out of range


def test_encoder_argument_errors():
    lib = _lib.load()
    v = np.zeros(10, dtype=np.uint32)
    out = np.zeros(1024, dtype=np.uint32)
    assert lib.scan_encode_for(v.ctypes.data, 10, 0, 0, 0, out.ctypes.data, None, None, None) == _lib.SCAN_EINVAL
    assert lib.scan_encode_for(v.ctypes.data, 10, 33, 0, 0, out.ctypes.data, None, None, None) == _lib.SCAN_EINVAL
    assert lib.scan_encode_for(v.ctypes.data, 10, 8, 2, 0, out.ctypes.data, None, None, None) == _lib.SCAN_EINVAL
    assert lib.scan_encode_for(v.ctypes.data, 10, 8, 0, 1, out.ctypes.data, None, None, None) == _lib.SCAN_EINVAL
    assert lib.scan_encode_dict(v.ctypes.data, 10, 3, 9, out.ctypes.data, None, None) == _lib.SCAN_EINVAL
    assert lib.scan_payload_words(0, 5) == 0 and lib.scan_payload_words(1025, 5) == 2 * 32 * 5


def test_block_sums_match_numpy(rng):
    """scan_block_sums (library host code) against per-block numpy sums mod 2^64."""
    for n in (1, 1023, 1024, 3 * 1024 + 17):
        v = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
        want = [int(v[k:k + 1024].astype(np.uint64).sum()) % (1 << 64) for k in range(0, n, 1024)]
        assert api.host_block_sums(api.ENC_FOR, v).tolist() == want
        d = np.cumsum(rng.integers(0, 1 << 20, size=n)).astype(np.int64) - (1 << 40)
        want = [sum(int(x) for x in d[k:k + 1024]) % (1 << 64) for k in range(0, n, 1024)]
        assert api.host_block_sums(api.ENC_DELTA, d).tolist() == want
        dct = np.sort(rng.choice(np.arange(-(1 << 40), 1 << 40, 1 << 28), size=300, replace=False)).astype(np.int64)
        codes = rng.integers(0, 300, size=n).astype(np.uint32)
        want = [sum(int(dct[c]) for c in codes[k:k + 1024]) % (1 << 64) for k in range(0, n, 1024)]
        assert api.host_block_sums(api.ENC_DICT, codes, dct).tolist() == want
    with pytest.raises(_lib.ScanError):
        api.host_block_sums(api.ENC_DICT, np.array([0, 300], dtype=np.uint32), np.arange(300, dtype=np.int64))


def test_rle_encoder_matches_oracle(rng):
    """The library's run-length encoder and the oracle's give identical arrays."""
    for n in (0, 1, 1023, 1025, 6000):
        for v in (np.repeat(rng.integers(0, 100, size=n // 5 + 1), 5)[:n].astype(np.uint32),
                  rng.integers(0, 2, size=n).astype(np.uint32)):
            rv, rl, br, zmin, zmax = api.host_encode_rle(v)
            orv, orl, obr = oracle.rle_encode(v)
            assert np.array_equal(rv, orv) and np.array_equal(rl, orl) and np.array_equal(br, obr)
            if n:
                omin, omax = oracle.zonemap_u32(v)
                assert np.array_equal(zmin, omin) and np.array_equal(zmax, omax)
