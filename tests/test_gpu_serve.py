"""GPU parity of conjunctive multi-column queries and of the query server.

A table shaped like the serving workload (FOR and dictionary columns of
widths 4..20, clustered and random halves) with a ragged row count; queries
with 1..3 conjuncts drawn like the workload's plus edge cases.  Every result
must equal the CPU oracle bit for bit, alone, in a batch and through the
server."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2606_22423_amd import _lib, api, serve  # noqa: E402

N = 37 * 1024 + 501


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def world(ctx):
    spec = synth.config5_table(10)
    cols, ocols, dicts, zones = [], [], {}, []
    for tc in spec:
        vals, dct = synth.config5_column(tc, N, s=64)
        if tc.enc == 0:
            cols.append(api.encode_for(vals, tc.b))
        else:
            cols.append(api.encode_dict(vals, tc.b, dct))
            dicts[tc.index] = dct
        ocols.append({"enc": tc.enc, "b": tc.b, "payload": oracle.pack_rm(vals, tc.b), "refs": None, "dict": dct})
        zones.append(oracle.zonemap_u32(vals))
    table = serve.Table(ctx, cols)
    qs = synth.config5_queries(120, spec, 1000.0, dicts)
    queries = [(q.filters, q.sum_col) for q in qs]
    d1 = dicts[1]
    queries += [
        ([(0, 5, 5)], 2),                                   # empty conjunct
        ([(0, 0, 1 << 32)], 0),                             # everything, sum of the filter column itself
        ([(2, -(1 << 40), 1 << 40), (4, 0, 9)], 3),         # clamped range plus a narrow one
        ([(1, int(d1[3]), int(d1[3]) + 1)], 5),             # dictionary equality
        ([(1, int(d1[0]) - 100, int(d1[0]))], 6),           # dictionary range with no entry
        ([(3, int(dicts[3][0]), int(dicts[3][-1]) + 1), (5, int(dicts[5][2]), int(dicts[5][-3])),
          (8, 0, 1 << 10)], 9),                             # three conjuncts
    ]
    yield {"table": table, "queries": queries, "ocols": ocols, "spec": spec, "zones": zones, "dicts": dicts}
    table.close()


def want(w, filters, sum_col):
    return oracle.query(w["ocols"], N, filters, sum_col)


def blocks_read(w, filters):
    """Blocks no conjunct's zone map excludes (zone maps in value or code domain)."""
    nb = (N + 1023) // 1024
    live = np.ones(nb, dtype=bool)
    for c, lo, hi in filters:
        zmin, zmax = w["zones"][c]
        if w["spec"][c].enc == 2:
            d = w["dicts"][c]
            lo, hi = int(np.searchsorted(d, lo)), int(np.searchsorted(d, hi))
        else:
            lo, hi = max(lo, 0), min(hi, 1 << 32)
        if lo >= hi:
            return 0
        live &= ~((zmax.astype(np.int64) < lo) | (zmin.astype(np.int64) >= hi))
    return int(live.sum())


def check(w, q, got):
    filters, sum_col = q
    r = want(w, filters, sum_col)
    assert got["status"] == 0, got
    assert (got["count"], got["sum"]) == (r.count, r.sum), (q, got, r)
    assert got["blocks_read"] == blocks_read(w, filters), (q, got)


KERNELS = [serve.SHARED, serve.PER_QUERY]


@pytest.fixture(params=KERNELS, ids=["shared", "per_query"])
def kernel(ctx, request):
    assert ctx.lib.scan_query_set_kernel(ctx.h, request.param) == 0
    yield request.param
    ctx.lib.scan_query_set_kernel(ctx.h, serve.PER_QUERY)


def test_batch_of_queries_matches_oracle(world, kernel):
    say("queries:", len(world["queries"]), "kernel", kernel)
    res = world["table"].run(world["queries"])
    for q, got in zip(world["queries"], res):
        check(world, q, got)


def test_each_result_is_the_same_alone_and_in_the_mix(world, kernel):
    mix = world["table"].run(world["queries"])
    for q, m in zip(world["queries"][:40], mix[:40]):
        alone = world["table"].run([q])[0]
        assert (alone["count"], alone["sum"], alone["blocks_read"]) == (m["count"], m["sum"], m["blocks_read"])


def test_launch_shape_does_not_change_results(ctx, world, kernel):
    base = world["table"].run(world["queries"][:70])
    try:
        for per_cu, win in ((1, 1), (4, 7), (8, 32)):
            ctx.lib.scan_query_set_tune(ctx.h, per_cu, win)
            got = world["table"].run(world["queries"][:70])
            assert [(g["count"], g["sum"], g["blocks_read"]) for g in got] == \
                [(b["count"], b["sum"], b["blocks_read"]) for b in base]
    finally:
        ctx.lib.scan_query_set_tune(ctx.h, 0, 0)


def test_kernel_choice_errors(ctx):
    assert ctx.lib.scan_query_set_kernel(ctx.h, 2) == _lib.SCAN_EINVAL  # neither kernel
    assert ctx.lib.scan_query_set_kernel(ctx.h, -1) == _lib.SCAN_EINVAL


def test_queries_at_2p22_rows_match_oracle(ctx):
    """The serving workload's table and queries at 2^22 rows (16 columns,
    widths 4..20, FOR and dictionary, half clustered): every result of a
    64-query batch equals the oracle, with both kernels."""
    n = 1 << 22
    spec = synth.config5_table(16)
    cols, ocols, dicts = [], [], {}
    for tc in spec:
        vals, dct = synth.config5_column(tc, n)
        cols.append(api.encode_for(vals, tc.b) if tc.enc == 0 else api.encode_dict(vals, tc.b, dct))
        if tc.enc != 0:
            dicts[tc.index] = dct
        ocols.append({"enc": tc.enc, "b": tc.b, "payload": oracle.pack_rm(vals, tc.b), "refs": None, "dict": dct})
    table = serve.Table(ctx, cols)
    try:
        qs = synth.config5_queries(64, spec, 1000.0, dicts, seed_stream=31)
        queries = [(q.filters, q.sum_col) for q in qs]
        wants = [oracle.query(ocols, n, f, s) for f, s in queries]
        for k in KERNELS:
            assert ctx.lib.scan_query_set_kernel(ctx.h, k) == 0
            say("2^22-row table, kernel", k)
            got = table.run(queries)
            for q, g, r in zip(queries, got, wants):
                assert (g["count"], g["sum"]) == (r.count, r.sum), (k, q, g, r)
    finally:
        ctx.lib.scan_query_set_kernel(ctx.h, serve.PER_QUERY)
        table.close()


def test_invalid_queries_are_rejected(world):
    with pytest.raises(_lib.ScanError):
        world["table"].run([([(99, 0, 1)], 0)])
    with pytest.raises(_lib.ScanError):
        world["table"].run([([], 0)])


@pytest.mark.parametrize("kern", KERNELS, ids=["shared", "per_query"])
def test_server_results_match_oracle(ctx, world, kern):
    srv = serve.Server(ctx, world["table"], serve.config(max_inflight=16, n_streams=2, max_batch=8,
                                                         batch_window_us=100, kernel=kern))
    try:
        tickets, results, busy = {}, {}, 0
        t0 = time.time()
        for i, (filters, s) in enumerate(world["queries"]):
            while True:
                tk = srv.submit(filters, s)
                if tk is not None:
                    tickets[tk] = i
                    break
                busy += 1
                for r in srv.poll(wait_us=1000):
                    results[r["ticket"]] = r
            assert time.time() - t0 < 60
        while len(results) < len(tickets):
            for r in srv.poll(wait_us=20000):
                results[r["ticket"]] = r
            assert time.time() - t0 < 60
        st = srv.stats()
    finally:
        srv.close()
    say("server: %d queries, %d refused submissions, %s" % (len(tickets), busy, st))
    assert st["launched"] == len(tickets) and st["inflight"] == 0
    for tk, i in tickets.items():
        r = results[tk]
        check(world, world["queries"][i], r)
        assert r["done_us"] >= r["submit_us"]
