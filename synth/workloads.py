"""Column and predicate recipes for the five measured workloads.

Each recipe returns raw column values (uint32 for frame-of-reference columns,
int64 for delta and dictionary columns, dictionary codes as uint32) plus
half-open predicate bounds [lo, hi).  Seeds: workload k uses
SEED_BASE + (k - 1); the PCG stream is the column index.

Nothing here encodes, decodes or scans; expected results come from the oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import SEED_BASE, bounded, gauss, pcg32, unit

__all__ = [
    "SIGMAS_SWEEP", "width_values", "lt_bound", "config1", "config2_draws", "config2_column",
    "noisy_perm", "config3_column", "config3_predicate", "ColumnSpec", "config4_specs",
    "config4_values", "dict_entries", "TableColumn", "config5_table", "config5_column",
    "Query", "config5_queries",
]

SIGMAS_SWEEP = (1e-4, 1e-3, 1e-2, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99)


def width_values(draws: np.ndarray, b: int) -> np.ndarray:
    """The top b bits of each 32-bit draw: uniform in [0, 2^b)."""
    if not 1 <= b <= 32:
        raise ValueError("b must be in 1..32")
    return draws if b == 32 else (draws >> np.uint32(32 - b)).astype(np.uint32)


def lt_bound(sigma: float, b: int) -> int:
    """c for the predicate v < c on uniform [0, 2^b) data: round(sigma 2^b) clamped to [1, 2^b]."""
    return int(min(max(round(sigma * (1 << b)), 1), 1 << b))


# ---------------------------------------------------------------- workload 1
def config1(n: int = 1 << 20):
    """N uniform values in [0, 2^8) (top 8 bits of PCG32), predicate v < 26."""
    v = width_values(pcg32(SEED_BASE, 0, n), 8)
    return v, 0, 26


# ---------------------------------------------------------------- workload 2
def config2_draws(n: int = 1 << 28) -> np.ndarray:
    """One PCG32 stream serves every width: the column at width b is draws >> (32-b)."""
    return pcg32(SEED_BASE + 1, 0, n)


def config2_column(draws: np.ndarray, b: int) -> np.ndarray:
    return width_values(draws, b)


# ---------------------------------------------------------------- workload 3
def noisy_perm(n: int, s, seed: int, stream: int, device: str = "cpu"):
    """Order of ranks 0..n-1 after displacing rank r to key r + round(s * z_r).

    z_r are Box-Muller normals clipped to |z| <= 8; ties keep rank order (stable
    sort).  s = 0 is the identity; s = "random" sorts by independent 64-bit
    uniform keys instead (a uniformly random permutation up to key ties).
    Returns a torch int64 tensor on ``device``: element i is the rank placed at
    position i.
    """
    import torch

    if s == 0:
        return torch.arange(n, dtype=torch.int64, device=device)
    if s == "random":
        hi = pcg32(seed, stream, n).astype(np.int64) << np.int64(31)
        lo = (pcg32(seed, stream + (1 << 32), n) >> np.uint32(1)).astype(np.int64)
        keys_np = hi | lo
    else:
        z = gauss(seed, stream, n, clip=8.0)
        keys_np = np.arange(n, dtype=np.int64) + np.rint(float(s) * z).astype(np.int64)
        del z
    keys = torch.from_numpy(keys_np).to(device)
    del keys_np
    _, order = torch.sort(keys, stable=True)
    return order


def config3_column(n: int = 1 << 30, n_distinct: int = 1 << 16, s=0, device: str = "cpu"):
    """Sorted base v_r = r * n_distinct / n (each value fills n / n_distinct
    consecutive ranks), displaced by the clustering knob s (see noisy_perm).
    Every level is a permutation of the same multiset.  Returns a uint32 torch
    tensor on ``device``."""
    import torch

    if n % n_distinct:
        raise ValueError("n must be a multiple of n_distinct")
    shift = int(math.log2(n // n_distinct))
    if (1 << shift) * n_distinct != n:
        raise ValueError("n / n_distinct must be a power of two")
    stream = {0: 0, 16: 1, 1024: 2, 65536: 3, "random": 4}.get(s, 5 + (int(s) if s != "random" else 0))
    order = noisy_perm(n, s, SEED_BASE + 2, stream, device=device)
    vals = (order >> shift).to(torch.int32)
    del order
    return vals.view(torch.uint32) if hasattr(torch, "uint32") else vals


def config3_predicate(sigma: float, n_distinct: int = 1 << 16, draw: int = 0):
    """[lo, lo + w) with w = max(1, round(sigma * n_distinct)), lo uniform in [0, n_distinct - w]."""
    w = max(1, int(round(sigma * n_distinct)))
    u = unit(SEED_BASE + 2, 1000 + draw, 1)[0]
    lo = int(u * (n_distinct - w + 1))
    lo = min(lo, n_distinct - w)
    return lo, lo + w


# ---------------------------------------------------------------- workload 4
@dataclass
class ColumnSpec:
    index: int
    n: int
    b: int
    enc: int          # 0 frame-of-reference, 1 delta, 2 dictionary
    sigma: float
    u_pred: float     # uniform draw that places the predicate window
    seed: int = field(default=SEED_BASE + 3)


def config4_specs(ncols: int = 4096, seed: int = SEED_BASE + 3, log2_min: float = 10.0,
                  log2_max: float = 24.0, bmax: int = 24, sigma_min: float = 1e-4,
                  sigma_max: float = 0.9, meta_stream: int = 1 << 40):
    """Per-column shape: n = floor(2^(log2_min + (log2_max-log2_min) u)), b uniform
    in 1..bmax, encoding = index mod 3, sigma log-uniform in [sigma_min, sigma_max]."""
    meta = unit(seed, meta_stream, 4 * ncols).reshape(ncols, 4)
    specs = []
    lmin, lmax = math.log10(sigma_min), math.log10(sigma_max)
    for i in range(ncols):
        u0, u1, u2, u3 = meta[i]
        n = int(math.floor(2.0 ** (log2_min + (log2_max - log2_min) * u0)))
        b = 1 + min(bmax - 1, int(u1 * bmax))
        sigma = 10.0 ** (lmin + (lmax - lmin) * u2)
        specs.append(ColumnSpec(i, n, b, i % 3, sigma, float(u3), seed))
    return specs


def dict_entries(m: int, seed: int, stream: int, half_range_log2: int) -> np.ndarray:
    """m strictly increasing int64 entries in [-2^h, 2^h): stratified, one per
    equal slice of the range, each at a bounded random offset inside its slice."""
    span = 1 << (half_range_log2 + 1)
    step = span // m
    jitter = bounded(seed, stream, m, min(step, 2**32 - 1)).astype(np.int64)
    return (-(1 << half_range_log2) + np.arange(m, dtype=np.int64) * step + jitter).astype(np.int64)


def config4_values(spec: ColumnSpec):
    """Raw values of one workload-4 column and its predicate.

    Returns (values, lo, hi, dictionary) where values are uint32 for
    frame-of-reference, int64 for delta, uint32 codes for dictionary (the
    dictionary entries are returned separately, sorted int64)."""
    n, b = spec.n, spec.b
    draws = pcg32(spec.seed, spec.index, n)
    if spec.enc == 0:
        v = width_values(draws, b)
        w = max(1, int(round(spec.sigma * (1 << b))))
        w = min(w, 1 << b)
        lo = min(int(spec.u_pred * ((1 << b) - w + 1)), (1 << b) - w)
        return v, lo, lo + w, None
    if spec.enc == 1:
        d = width_values(draws, b).astype(np.int64)
        d[0] = int(draws[0])  # first value: uniform in [0, 2^32)
        v = np.cumsum(d, dtype=np.int64)
        p = min(int(spec.u_pred * n), n - 1)
        q = p + int(math.ceil(spec.sigma * n))
        lo = int(v[p])
        hi = int(v[q]) if q < n else int(v[-1]) + 1
        return v, lo, hi, None
    m = min(1 << b, 4096)
    dct = dict_entries(m, spec.seed, spec.index + (1 << 33), 38)
    codes = width_values(draws, b) if (1 << b) <= 4096 else bounded(spec.seed, spec.index + (1 << 34), n, m)
    cw = max(1, int(round(spec.sigma * m)))
    cw = min(cw, m)
    clo = min(int(spec.u_pred * (m - cw + 1)), m - cw)
    lo = int(dct[clo])
    hi = int(dct[clo + cw]) if clo + cw < m else int(dct[-1]) + 1
    return codes.astype(np.uint32), lo, hi, dct


# ---------------------------------------------------------------- workload 5
@dataclass
class TableColumn:
    index: int
    b: int
    enc: int          # 0 frame-of-reference, 2 dictionary
    clustered: bool
    m: int = 0        # dictionary size


def config5_table(ncols: int = 16):
    cols = []
    for j in range(ncols):
        b = (4, 8, 12, 16, 20)[j % 5]
        enc = 0 if j % 2 == 0 else 2
        m = min(1 << b, 4096) if enc == 2 else 0
        cols.append(TableColumn(j, b, enc, j < ncols // 2, m))
    return cols


def config5_column(col: TableColumn, n: int, device: str = "cpu", s: int = 1024):
    """Values (FOR, uint32) or codes (dictionary, uint32) plus dictionary entries.

    Clustered columns permute a sorted base by the noisy order with std s ranks;
    the others are uniform draws.  Returns (numpy uint32 array, entries or None)."""
    seed = SEED_BASE + 4
    dom = (1 << col.b) if col.enc == 0 else col.m
    if col.clustered:
        order = noisy_perm(n, s, seed, 100 + col.index, device=device).cpu().numpy()
        vals = ((order.astype(np.uint64) * np.uint64(dom)) // np.uint64(n)).astype(np.uint32)
        del order
    else:
        draws = pcg32(seed, col.index, n)
        if dom == (1 << col.b):
            vals = width_values(draws, col.b)
        else:
            vals = bounded(seed, col.index + (1 << 34), n, dom)
    dct = dict_entries(col.m, seed, col.index + (1 << 33), 34) if col.enc == 2 else None
    return vals, dct


@dataclass
class Query:
    qid: int
    filters: list      # [(column index, lo, hi)], 1..3 conjuncts over distinct columns
    sum_col: int
    arrival: float     # seconds since start (Poisson process)


def config5_queries(nq: int, table, rate_qps: float, dicts: dict, seed_stream: int = 7,
                    sigma_min: float = 1e-5, sigma_max: float = 0.5):
    """Poisson arrivals at rate_qps; m ~ U{1,2,3} distinct filter columns plus a
    distinct SUM column; each conjunct's sigma is log-uniform in [sigma_min, sigma_max]
    and its window width is rounded as for workload 4 (value domain 2^b for
    frame-of-reference, dictionary size for dictionary columns)."""
    seed = SEED_BASE + 4
    ncols = len(table)
    u = unit(seed, (1 << 36) + seed_stream, nq * 12).reshape(nq, 12)
    lmin, lmax = math.log10(sigma_min), math.log10(sigma_max)
    t = 0.0
    out = []
    for q in range(nq):
        r = u[q]
        t += -math.log(r[0]) / rate_qps
        m = 1 + min(2, int(r[1] * 3))
        # choose m+1 distinct columns by a partial Fisher-Yates over the column ids
        ids = list(range(ncols))
        picks = []
        for k in range(m + 1):
            j = k + min(ncols - k - 1, int(r[2 + k] * (ncols - k)))
            ids[k], ids[j] = ids[j], ids[k]
            picks.append(ids[k])
        filters = []
        for k in range(m):
            col = table[picks[k]]
            sigma = 10.0 ** (lmin + (lmax - lmin) * r[6 + k])
            if col.enc == 0:
                dom = 1 << col.b
                w = min(dom, max(1, int(round(sigma * dom))))
                lo = min(int(r[9 + k] * (dom - w + 1)), dom - w)
                filters.append((col.index, lo, lo + w))
            else:
                dct = dicts[col.index]
                mm = len(dct)
                w = min(mm, max(1, int(round(sigma * mm))))
                clo = min(int(r[9 + k] * (mm - w + 1)), mm - w)
                lo = int(dct[clo])
                hi = int(dct[clo + w]) if clo + w < mm else int(dct[-1]) + 1
                filters.append((col.index, lo, hi))
        out.append(Query(q, filters, picks[m], t))
    return out
