"""Pins of the shared input generators (no method arithmetic lives there)."""
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_pcg32_known_answers():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "pcg32_seed42_stream54.txt"))
            if l.strip() and not l.startswith("#")]
    got = synth.pcg32(42, 54, len(want))
    assert [int(x) for x in got] == want


def test_pcg32_jump_ahead_is_offset_independent():
    a = synth.pcg32(7, 3, 300_001)
    b = np.concatenate([synth.pcg32(7, 3, 123_456), synth.pcg32(7, 3, 300_001 - 123_456, offset=123_456)])
    assert np.array_equal(a, b)
    assert not np.array_equal(synth.pcg32(7, 3, 1000), synth.pcg32(7, 4, 1000))


def test_bounded_and_unit_ranges():
    x = synth.bounded(1, 2, 100_000, 10)
    assert x.min() == 0 and x.max() == 9
    # multiply-shift on the same draws: floor(draw * range / 2^32)
    d = synth.pcg32(1, 2, 1000).astype(np.uint64)
    assert np.array_equal(synth.bounded(1, 2, 1000, 12345), (d * np.uint64(12345)) >> np.uint64(32))
    u = synth.unit(3, 4, 100_000)
    assert 0.0 < u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


def test_gauss_moments_and_clip():
    z = synth.gauss(5, 6, 400_000, clip=8.0)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert np.abs(synth.gauss(5, 6, 1000, clip=0.5)).max() <= 0.5


def test_fisher_yates_is_permutation():
    p = synth.fisher_yates(9, 1, 100_003)
    assert np.array_equal(np.sort(p), np.arange(100_003, dtype=np.uint32))
    assert not np.array_equal(p, np.arange(100_003, dtype=np.uint32))


def test_noisy_perm_permutation_and_locality():
    for s in (0, 16, 1024, "random"):
        p = synth.noisy_perm(1 << 16, s, 11, 2).numpy()
        assert np.array_equal(np.sort(p), np.arange(1 << 16))
        if s not in ("random",):
            # ranks move by at most 2 * 8 * s positions (keys clipped at |z| <= 8)
            assert np.abs(p - np.arange(1 << 16)).max() <= 16 * (s if s else 0) + 1


def test_config_recipes_shapes():
    v, lo, hi = synth.config1(1 << 12)
    assert v.dtype == np.uint32 and v.max() < 256 and (lo, hi) == (0, 26)
    specs = synth.config4_specs(64)
    assert all(1 << 10 <= s.n < 1 << 24 and 1 <= s.b <= 24 for s in specs)
    assert [s.enc for s in specs[:6]] == [0, 1, 2, 0, 1, 2]
    for s in specs[:9]:
        s.n = min(s.n, 5000)
        vals, lo, hi, d = synth.config4_values(s)
        assert lo < hi and len(vals) == s.n
        if s.enc == 1:
            assert np.all(np.diff(vals) >= 0) and np.all(np.diff(vals) < (1 << s.b))
        if s.enc == 2:
            assert np.all(np.diff(d) > 0) and vals.max() < len(d)
