"""Python face of the serving ABI: tables, batched conjunctive queries and the
continuous-batching server (argument marshalling only)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import ScanError, ScanQuery, ScanQueryResult, ScanServerConfig, ScanTableColumn


def make_query(filters, sum_col: int) -> ScanQuery:
    """filters: [(column, lo, hi)] (1..3 conjuncts)."""
    q = ScanQuery()
    q.n_filters = len(filters)
    for f, (c, lo, hi) in enumerate(filters):
        q.filter_col[f] = int(c)
        q.filter[f].lo = int(lo)
        q.filter[f].hi = int(hi)
    q.sum_col = int(sum_col)
    return q


PER_QUERY, SHARED = 0, 1  # query kernels (scan_query_set_kernel)


def config(hbm_budget_bytes=2 << 30, max_inflight=256, n_streams=2, max_batch=64, batch_window_us=200,
           window_blocks=0, wgs_per_cu=0, kernel=PER_QUERY) -> ScanServerConfig:
    return ScanServerConfig(int(hbm_budget_bytes), max_inflight, n_streams, max_batch, batch_window_us,
                            window_blocks, wgs_per_cu, kernel, 0)


class Table:
    """Columns (api.Column, FOR or dictionary, row-major, with zone maps) of equal length."""

    def __init__(self, ctx, columns):
        self.ctx = ctx
        self.columns = list(columns)  # keeps the device buffers alive
        arr = (ScanTableColumn * len(columns))()
        for i, c in enumerate(columns):
            arr[i] = ScanTableColumn(c.struct(True), c.enc, c.b)
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.scan_table_create(ctx.h, arr, len(columns), ctypes.byref(h)), "scan_table_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.scan_table_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, queries) -> list:
        """Run queries (ScanQuery or (filters, sum_col)) as one batch; list of result dicts."""
        qs = [q if isinstance(q, ScanQuery) else make_query(*q) for q in queries]
        arr = (ScanQuery * max(1, len(qs)))(*qs)
        out = (ScanQueryResult * max(1, len(qs)))()
        self.ctx.check(self.ctx.lib.scan_query_run(self.ctx.h, self.h, arr, len(qs), out), "scan_query_run")
        return [out[i].as_dict() for i in range(len(qs))]


class Server:
    def __init__(self, ctx, table: Table, cfg: ScanServerConfig | None = None):
        self.lib = ctx.lib
        self.table = table
        h = ctypes.c_void_p()
        ctx.check(self.lib.scan_server_create(ctx.h, table.h, ctypes.byref(cfg or config()), ctypes.byref(h)),
                  "scan_server_create")
        self.h = h

    def submit(self, filters, sum_col: int):
        """Ticket, or None when admission refused the query (SCAN_EBUSY)."""
        t = ctypes.c_uint64()
        rc = self.lib.scan_server_submit(self.h, ctypes.byref(make_query(filters, sum_col)), ctypes.byref(t))
        if rc == _lib.SCAN_EBUSY:
            return None
        if rc != 0:
            raise ScanError(rc, "scan_server_submit")
        return int(t.value)

    def poll(self, max_results: int = 1024, wait_us: int = 0) -> list:
        out = (ScanQueryResult * max_results)()
        n = ctypes.c_size_t()
        rc = self.lib.scan_server_poll(self.h, out, max_results, ctypes.byref(n), wait_us)
        if rc != 0:
            raise ScanError(rc, "scan_server_poll")
        return [out[i].as_dict() for i in range(n.value)]

    def stats(self) -> dict:
        s = (ctypes.c_uint64 * 4)()
        self.lib.scan_server_stats(self.h, s)
        return {"batches": int(s[0]), "launched": int(s[1]), "inflight": int(s[2]), "pending": int(s[3])}

    @staticmethod
    def clock_us() -> float:
        return float(_lib.load().scan_server_clock_us())

    def close(self):
        if getattr(self, "h", None):
            self.lib.scan_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(cfg: ScanServerConfig, arrivals_us, batch_fixed_us: float, per_query_us: float):
    """Host-only run of the server's admission and batching policy.

    Returns (launch_us, done_us, status) numpy arrays and the batch count."""
    lib = _lib.load()
    a = np.ascontiguousarray(arrivals_us, dtype=np.float64)
    n = len(a)
    launch = np.zeros(n)
    done = np.zeros(n)
    status = np.zeros(n, dtype=np.int32)
    nb = ctypes.c_uint64()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.scan_serve_simulate(ctypes.byref(cfg), a.ctypes.data_as(dp), n, batch_fixed_us, per_query_us,
                                 launch.ctypes.data_as(dp), done.ctypes.data_as(dp),
                                 status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nb))
    if rc != 0:
        raise ScanError(rc, "scan_serve_simulate")
    return launch, done, status, int(nb.value)
