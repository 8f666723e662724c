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


# ------------------------------------------------- zone maps and clustering
def _trunc_normal_pmf(s: float, clip: float):
    """pmf of D = round(s z) for z standard normal truncated to |z| <= clip,
    over the integers t = -T .. T (T = round(clip s)).  Returns (T, pmf)."""
    from scipy.special import ndtr  # standard normal CDF
    T = int(round(clip * s))
    t = np.arange(-T, T + 1, dtype=np.float64)
    lo = np.maximum((t - 0.5) / s, -clip)
    hi = np.minimum((t + 0.5) / s, clip)
    pmf = np.maximum(ndtr(hi) - ndtr(lo), 0.0)
    return T, pmf / pmf.sum()


def read_fraction_model(n: int, lo: int, hi: int, s, n_distinct: int = 1 << 16, L: int = 1024,
                        clip: float = 8.0) -> float:
    """Expected fraction of 1024-value blocks that zone maps keep for [lo, hi)
    on the clustered column of the zone-map workload: the sorted column
    v_r = r // P (P = n / n_distinct copies of each value) with rank r moved
    to position ~ r + D_r, D_r = round(s z_r) independent truncated normals
    (s = "random": a uniform permutation).

    The predicate covers the ranks [A, E) = [lo P, hi P).  A block's zone map
    misses it iff all its ranks are >= E or all are < A (disjoint events), so
        P(read k) = 1 - P(no rank < E lands in k) - P(no rank >= A lands in k),
    and with independent displacements, for the block's first position kL,
        P(no rank < E lands in k)  = prod_{d >= 1} (1 - q(kL - E + d)),
        P(no rank >= A lands in k) = prod_{d >= 0} (1 - q(kL - A - d)),
    q(y) = P(D in [y, y + L)).  Both products are tail / prefix sums of
    log(1 - q) over one integer grid, so every block costs O(1).  The random
    permutation gives P(read) = 1 - (A/n)^L - ((n - E)/n)^L (values drawn
    independently).  s = 0 is exact: the blocks overlapping [A, E).
    This is the skipping side of the paper's two crossovers (clustering, not
    selectivity, decides what zone maps save), made quantitative."""
    P = n // n_distinct
    nb = n // L
    A, E = lo * P, hi * P
    if A >= E:
        return 0.0
    if s == 0:
        return float(-(-E // L) - A // L) / nb
    if s == "random":
        p = 1.0 - (A / n) ** L - ((n - E) / n) ** L
        return float(max(p, 0.0))
    T, pmf = _trunc_normal_pmf(float(s), clip)
    # q(y) for y = -T - L + 1 .. T: window sums of the pmf
    cum = np.concatenate([[0.0], np.cumsum(pmf)])            # cum[i] = P(D < -T + i)
    y = np.arange(-T - L + 1, T + 1)
    a = np.clip(y + T, 0, 2 * T + 1)
    b = np.clip(y + L + T, 0, 2 * T + 1)
    q = np.clip(cum[b] - cum[a], 0.0, 1.0)
    with np.errstate(divide="ignore"):
        g = np.log1p(-q)
    g = np.where(q >= 1.0, -np.inf, g)
    y0 = int(y[0])
    # prefix and suffix sums kept apart (log(1 - q) is -inf where a window
    # holds the whole support, and -inf - -inf would be undefined)
    pre = np.concatenate([[0.0], np.cumsum(g)])              # pre[i] = sum g(y0 .. y0 + i - 1)
    suf = np.concatenate([np.cumsum(g[::-1])[::-1], [0.0]])  # suf[i] = sum g(y0 + i ..)

    def prefix(w):   # sum_{y <= w} g(y)
        return pre[np.clip(w - y0 + 1, 0, len(g))]

    def tail(v):     # sum_{y >= v} g(y)
        return suf[np.clip(v - y0, 0, len(g))]

    k0 = max(0, (A - T - 2 * L) // L)
    k1 = min(nb, (E + T + 2 * L) // L + 1)
    k = np.arange(k0, k1, dtype=np.int64)
    f_up = np.exp(tail(k * L - E + 1))
    f_dn = np.exp(prefix(k * L - A))
    p = np.clip(1.0 - f_up - f_dn, 0.0, 1.0)
    return float(p.sum()) / nb
