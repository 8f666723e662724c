"""The decode-throughput law and its one-parameter fit (host-side measurement logic).

The paper's model ("Problem and Model", the boxed law): reading N values of b
bits moves N*b/8 bytes, so the roofline floor is T >= N*b/(8*beta) and the
bandwidth fraction is f = (N*b/8 / T) / beta.  If a decoder produces T_dec
values per second whatever b is, then f = min(1, T_dec*b/(8*beta)) and the
compute-to-bandwidth ridge is b* = 8*beta/T_dec.  One T_dec is fitted per
decode strategy ("Results: the law"); the fit quality is the median |f - f_hat|.

The paper does not say how T_dec is fitted.  This module's reading: T_dec
minimises the squared error of the full law min(1, T b / (8 beta)) over all
measured widths, found on a dense log grid and refined.  (Minimising the
median error itself is degenerate: once more than half of the widths sit on
the plateau, a whole interval of T_dec scores zero.)  The paper's statistic,
the median |f - f_hat|, is reported for the fitted T_dec, and a least-squares
fit through the origin on the compute-bound points (f < 0.9) is reported
beside it as a cross-check.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def bandwidth_fraction(n_values: float, b: float, seconds: float, beta: float) -> float:
    """f = (N b / 8 / T) / beta."""
    return (n_values * b / 8.0 / seconds) / beta


def law(t_dec: float, b, beta: float):
    """f_hat = min(1, T_dec b / (8 beta)) (vectorised over b)."""
    return np.minimum(1.0, t_dec * np.asarray(b, dtype=np.float64) / (8.0 * beta))


def ridge(t_dec: float, beta: float) -> float:
    """b* = 8 beta / T_dec."""
    return 8.0 * beta / t_dec


def median_abs_error(t_dec: float, bs, fs, beta: float) -> float:
    return float(np.median(np.abs(np.asarray(fs, dtype=np.float64) - law(t_dec, bs, beta))))


@dataclass
class Fit:
    t_dec: float          # values/s
    b_star: float         # bits
    median_err: float
    t_dec_ls: float       # least squares on f < 0.9 points (nan if none)
    n_points: int
    compute_bound_points: int


def fit_tdec(bs, fs, beta: float, decades: tuple = (6.0, 15.0), per_decade: int = 1000) -> Fit:
    """Fit one T_dec (values/s) to measured (b, f) pairs against bandwidth beta (bytes/s)."""
    bs = np.asarray(bs, dtype=np.float64)
    fs = np.asarray(fs, dtype=np.float64)
    if len(bs) == 0 or len(bs) != len(fs):
        raise ValueError("need matching, non-empty b and f lists")
    def sse(t):
        return float(np.sum((np.minimum(1.0, t * bs / (8.0 * beta)) - fs) ** 2))

    grid = 10.0 ** np.linspace(decades[0], decades[1], int((decades[1] - decades[0]) * per_decade) + 1)
    pred = np.minimum(1.0, np.outer(grid, bs) / (8.0 * beta))
    err = np.sum((pred - fs[None, :]) ** 2, axis=1)
    i = int(np.argmin(err))
    # refine between the neighbouring grid points (ternary search; the objective
    # is unimodal in T there)
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    for _ in range(200):
        m1, m2 = lo + (hi - lo) / 3.0, hi - (hi - lo) / 3.0
        if sse(m1) <= sse(m2):
            hi = m2
        else:
            lo = m1
    t_best = min((sse(t), t) for t in (grid[i], 0.5 * (lo + hi)))[1]
    best_err = median_abs_error(t_best, bs, fs, beta)
    cb = fs < 0.9
    if cb.any():
        x = bs[cb] / (8.0 * beta)
        t_ls = float(np.sum(x * fs[cb]) / np.sum(x * x))
    else:
        t_ls = float("nan")
    return Fit(float(t_best), ridge(float(t_best), beta), float(best_err), t_ls, int(len(bs)), int(cb.sum()))


def sigma_achieved(c: int, b: int) -> float:
    """Selectivity of v < c on uniform [0, 2^b) data."""
    return c / float(1 << b)


def is_quantized(sigma_target: float, c: int, b: int) -> bool:
    """Flag widths where v < c cannot get within half a decade of the target selectivity."""
    return abs(math.log10(sigma_achieved(c, b) / sigma_target)) > 0.3


# ------------------------------------------------- branch-free vs compaction
@dataclass
class Crossover:
    a_bf: float           # seconds: branch-free cost model a + b * sigma
    b_bf: float
    a_sv: float           # selection-vector (compaction) cost model
    b_sv: float
    sigma_star: float     # where the two models meet (nan if they do not cross in (0, 1))
    faster_below: str     # mode that wins for sigma below sigma_star ("bf" or "sv"; the winner everywhere if no cross)


def _linear(x, y):
    """Least-squares line y = a + b x."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    b, a = np.polyfit(x, y, 1)
    return float(a), float(b)


def fit_crossover(sigmas, t_bf, t_sv) -> Crossover:
    """The GPU analogue of the paper's branchy / branch-free crossover.

    On a CPU the branchy filter pays A + B sigma (1 - sigma) for
    mispredictions ("Results: the two crossovers").  A wavefront has no
    branch predictor: the branch-free mode tests and masks every value, so its
    time is flat in sigma, while compaction writes each selected value to LDS
    and reads it back, so its time grows linearly with the selected count.
    Both are fitted as a + b sigma by least squares; sigma* solves
    a_bf + b_bf s = a_sv + b_sv s."""
    s = np.asarray(sigmas, dtype=np.float64)
    if len(s) < 2 or len(s) != len(t_bf) or len(s) != len(t_sv):
        raise ValueError("need at least two matching (sigma, t_bf, t_sv) points")
    a1, b1 = _linear(s, t_bf)
    a2, b2 = _linear(s, t_sv)
    star = float("nan")
    if b1 != b2:
        x = (a2 - a1) / (b1 - b2)
        if 0.0 < x < 1.0:
            star = float(x)
    low = 1e-6 if star != star else star * 0.5
    faster = "bf" if a1 + b1 * low <= a2 + b2 * low else "sv"
    return Crossover(a1, b1, a2, b2, star, faster)
