"""Pins of the law and its fit: synthetic recovery, the paper's Table 1
consistency, and the large-T_dec (FastLanes) limit the paper quotes."""
import os

import numpy as np
import pytest

from paper_2606_22423_amd import lawfit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def table1():
    rows = []
    for line in open(os.path.join(GOLDEN, "table1_fits.txt")):
        if line.strip() and not line.startswith("#"):
            m, s, t, b, e = line.split()
            rows.append((m, s, float(t), float(b), float(e)))
    return rows


@pytest.mark.parametrize("t_dec,beta", [(3.91e9, 14.3e9), (8.0e12, 6.9e12), (2.5e11, 7.1e12), (9.04e9, 70e9)])
def test_fit_recovers_synthetic_law(t_dec, beta):
    bs = np.arange(1, 33)
    fs = lawfit.law(t_dec, bs, beta)
    fit = lawfit.fit_tdec(bs, fs, beta)
    if np.all(fs >= 1.0):
        pytest.skip("every point on the plateau: T_dec is unidentifiable")
    assert abs(fit.t_dec / t_dec - 1) < 1e-6
    assert abs(fit.b_star / lawfit.ridge(t_dec, beta) - 1) < 1e-6
    assert fit.median_err < 1e-9
    if fit.compute_bound_points:
        assert abs(fit.t_dec_ls / t_dec - 1) < 1e-9


def test_fit_with_noise_and_plateau():
    rng = np.random.default_rng(3)
    beta, t = 7.0e12, 9.0e12
    bs = np.arange(1, 33)
    fs = lawfit.law(t, bs, beta) * (1 + 0.01 * rng.standard_normal(32))
    fit = lawfit.fit_tdec(bs, fs, beta)
    assert abs(fit.t_dec / t - 1) < 0.03 and fit.median_err < 0.02


def test_table1_is_consistent_with_the_stated_bandwidths():
    for machine, strategy, t_dec, b_star, _ in table1():
        beta = b_star * t_dec / 8.0  # GB/s
        if machine == "x86":
            assert 14.0 <= beta <= 16.0, (strategy, beta)
        else:
            assert 69.5 <= beta <= 70.5, (strategy, beta)
        assert abs(lawfit.ridge(t_dec * 1e9, beta * 1e9) - b_star) < 1e-9


def test_large_tdec_limit_reproduces_decode_is_free_at_three_bits():
    """T_dec = 140 Gval/s against 52 GB/s: f(3) = 1 and the ridge is 2.97 bits."""
    t, beta = 140e9, 52e9
    assert lawfit.law(t, 3, beta) == 1.0
    assert abs(lawfit.ridge(t, beta) - 8 * 52 / 140) < 1e-12
    assert lawfit.law(t, 2, beta) < 1.0


def test_bandwidth_fraction_and_quantization():
    assert lawfit.bandwidth_fraction(2**28, 8, 2**28 / 7e12, 7e12) == pytest.approx(1.0)
    assert lawfit.sigma_achieved(1, 1) == 0.5
    assert lawfit.is_quantized(1e-4, 1, 1) and not lawfit.is_quantized(0.1, 6554, 16)


def test_crossover_recovers_synthetic_lines():
    s = np.array([1e-4, 1e-3, 1e-2, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99])
    # compaction cheaper at low selectivity, branch-free flat
    t_bf = 1.0 + 0.0 * s
    t_sv = 0.6 + 0.8 * s
    c = lawfit.fit_crossover(s, t_bf, t_sv)
    assert c.sigma_star == pytest.approx(0.5, abs=1e-9)
    assert c.faster_below == "sv"
    assert (c.a_bf, c.b_bf) == pytest.approx((1.0, 0.0), abs=1e-9)
    assert (c.a_sv, c.b_sv) == pytest.approx((0.6, 0.8), abs=1e-9)


def test_crossover_absent_when_one_mode_always_wins():
    s = np.linspace(0.0, 1.0, 11)
    c = lawfit.fit_crossover(s, 1.0 + 0.01 * s, 1.5 + 0.5 * s)
    assert c.sigma_star != c.sigma_star  # nan: no crossing in (0, 1)
    assert c.faster_below == "bf"
    with pytest.raises(ValueError):
        lawfit.fit_crossover([0.1], [1.0], [2.0])


@pytest.mark.parametrize("s", [0, 16, 1024, 65536, "random"])
def test_read_fraction_model_matches_generated_columns(s):
    """The clustering model of the zone-map workload (expected share of blocks
    the zone maps keep) against exact counts on columns drawn by the
    workload's own generator at 2^22 values (each value fills 64 ranks): within
    3 blocks + 3 % of the count for every (selectivity, predicate draw)."""
    import oracle
    import synth
    n = 1 << 22
    v = synth.config3_column(n, s=s).numpy().view(np.uint32)
    zmin, zmax = oracle.zonemap_u32(v)
    for sg in (1e-4, 1e-3, 1e-2, 0.1, 0.5):
        for draw in range(2):
            lo, hi = synth.config3_predicate(sg, draw=draw)
            meas = int(np.sum(~((zmax < lo) | (zmin >= hi))))
            model = lawfit.read_fraction_model(n, lo, hi, s) * (n // 1024)
            assert abs(meas - model) <= 3 + 0.03 * model, (s, sg, draw, meas, model)
            if s == 0:
                assert meas == round(model)


def test_read_fraction_model_limits():
    """Closed limits: an empty predicate reads nothing; the sorted column reads
    exactly the blocks its value range covers; the random permutation follows
    1 - (lo/V)^L - ((V-hi)/V)^L; a small displacement (s << L) adds at most
    one block per predicate edge."""
    n, V = 1 << 30, 1 << 16
    assert lawfit.read_fraction_model(n, 10, 10, 1024) == 0.0
    assert lawfit.read_fraction_model(n, 100, 107, 0) * (n // 1024) == 7 * 16
    lo, hi = 1000, 1007
    want = 1 - (lo / V) ** 1024 - ((V - hi) / V) ** 1024
    assert abs(lawfit.read_fraction_model(n, lo, hi, "random") - want) < 1e-12
    extra = lawfit.read_fraction_model(n, lo, hi, 4) * (n // 1024) - 7 * 16
    assert 0.0 <= extra <= 2.0 + 1e-9
