"""Fixed workload for rocprofv3 runs of the hot path's kernels beyond the
frame-of-reference sweep: dictionary and delta scans, the batch class
kernels, the serving query kernel, the run-length scan and the materializing
select's passes.  Each case launches its kernels a few times on a cold cache
(a 512 MiB read of scratch before each launch) and reports its algorithmic
bytes per launch; calibration kernels of known traffic (a 1 GiB streaming
read, a triad) run first for the HBM byte counters.

    rocprofv3 --kernel-trace --stats -- python3 -m paper_2606_22423_amd.profile_paths
    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2606_22423_amd.profile_paths

Prints one JSON line: {"cases": [{"name", "kernel", "launches",
"algorithmic_bytes", "values", ...}], "cal_read_bytes", "cal_triad_floats"}.
`kernel` is a regular expression on the kernel names of the trace.
"""
from __future__ import annotations

import argparse
import json
import sys

CAL_READ_BYTES = 1 << 30
CAL_TRIAD_FLOATS = 1 << 26


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-log2", type=int, default=28)
    ap.add_argument("--launches", type=int, default=5)
    ap.add_argument("--skip", default="", help="comma-separated case families to leave out")
    args = ap.parse_args(argv)
    skip = set(filter(None, args.skip.split(",")))

    import numpy as np
    import torch

    import synth
    from paper_2606_22423_amd import api, serve
    from paper_2606_22423_amd import selector_train as st
    from paper_2606_22423_amd._lib import DEC_RM_DIRECT, DEC_RM_LDS, strategy

    say = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    ctx = api.Context(0)
    buf = torch.empty(CAL_READ_BYTES // 4, dtype=torch.int32, device="cuda")
    buf.fill_(1)
    sink = torch.zeros(16, dtype=torch.int64, device="cuda")
    for _ in range(3):
        ctx.beta_read(buf, CAL_READ_BYTES, sink)
    a = torch.empty(CAL_TRIAD_FLOATS, device="cuda")
    b = torch.ones(CAL_TRIAD_FLOATS, device="cuda")
    c = torch.ones(CAL_TRIAD_FLOATS, device="cuda")
    for _ in range(3):
        ctx.beta_triad(a, b, c, 2.0)
    torch.cuda.synchronize()
    del buf, a, b, c
    evict = torch.empty(512 << 18, dtype=torch.int32, device="cuda")
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    n = 1 << args.n_log2
    cases = []

    def flush():
        ctx.cache_flush(evict, evict.numel() * 4)

    def timed(fn):
        evs = []
        for _ in range(args.launches):
            flush()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ms = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
        return ms[len(ms) // 2]

    draws = synth.config2_draws(n)
    dec_names = {DEC_RM_LDS: "rm_lds", DEC_RM_DIRECT: "rm_direct"}
    # --- dictionary scans: 2^b sorted int64 entries, codes uniform, 10 % of the codes selected
    if "dict" not in skip:
        for b in (4, 8, 12):
            m = 1 << b
            dct = synth.dict_entries(m, synth.SEED_BASE + 1, 1 << 35, 38)
            codes = synth.config2_column(draws, b)
            cw = max(1, round(0.1 * m))
            clo = (m - cw) // 2
            lo, hi = int(dct[clo]), int(dct[clo + cw])
            col = api.encode_dict(codes, b, dct, block_sums=False)
            del codes
            for dec in (DEC_RM_DIRECT, DEC_RM_LDS):
                s = strategy(dec, 0, 0)
                ms = timed(lambda: ctx.run_async(col, lo, hi, s, out))
                cases.append({"name": "dictionary b=%d %s/bf/nozm" % (b, dec_names[dec]),
                              "kernel": r"code_scan<%d, %d, 0, 2, \d+(, \d+)?>" % (b, dec), "launches": args.launches,
                              "algorithmic_bytes": n * b // 8, "values": n, "event_ms": ms})
            del col
            say("dictionary b=%d done" % b)
    # --- delta scans: cumulative sums of b-bit draws
    if "delta" not in skip:
        for b in (8, 16, 24):
            d = synth.config2_column(draws, b).astype(np.int64)
            v = np.cumsum(d, dtype=np.int64)
            del d
            lo, hi = int(v[int(0.45 * n)]), int(v[int(0.55 * n)])
            col = api.encode_delta(v, b, block_sums=False)
            del v
            for dec in (DEC_RM_DIRECT, DEC_RM_LDS):
                s = strategy(dec, 0, 0)
                ms = timed(lambda: ctx.run_async(col, lo, hi, s, out))
                cases.append({"name": "delta b=%d %s/bf/nozm" % (b, dec_names[dec]),
                              "kernel": r"delta_scan<%d, %d, 0>" % (b, dec), "launches": args.launches,
                              "algorithmic_bytes": n * b // 8 + (n // 1024) * 8, "values": n, "event_ms": ms})
            del col
            say("delta b=%d done" % b)
    del draws
    # --- batch class kernels: the 4096-column mixed workload, default strategy
    if "batch" not in skip:
        specs = synth.config4_specs(4096)
        cols = st.build_columns(specs)
        default = strategy(DEC_RM_DIRECT, 0, 1)
        items = [c.item(lo, hi, default) for c, lo, hi in cols]
        h = ctx.batch_prepare(items)
        res = ctx.batch_replay(h, len(items))
        ms = timed(lambda: ctx.batch_replay(h, wait=False))
        ctx.batch_release(h)
        per = {}
        for (c, lo, hi), sp, r in zip(cols, specs, res):
            zm_bytes = (16 if sp.enc == 1 else 8) * ((sp.n + 1023) // 1024)
            byt = r["blocks_read"] * 128 * sp.b + zm_bytes
            if sp.enc == 2 and r["blocks_read"]:
                byt += 8 * c.dct.numel()
            key = (sp.enc, 1, 0)
            per.setdefault(key, [0, 0])
            per[key][0] += byt
            per[key][1] += r["blocks_read"] * 1024
        enc_names = {0: "FOR", 1: "delta", 2: "dictionary"}
        for (enc, dec, mode), (byt, vals) in sorted(per.items()):
            cases.append({"name": "batch class %s rm_direct/bf (4096-column workload, zone maps)" % enc_names[enc],
                          "kernel": r"batch_scan<%d, %d, %d>" % (enc, dec, mode), "launches": args.launches + 1, "warmup": 1,
                          "algorithmic_bytes": int(byt), "values": int(vals), "event_ms": ms})
        del cols
        say("batch done")
    # --- serving query kernel: 16 columns x 2^n rows, one batch of 64 queries
    if "serve" not in skip:
        spec = synth.config5_table(16)
        tcols, dicts = [], {}
        for tc in spec:
            vals, dct = synth.config5_column(tc, n, device="cuda")
            tcols.append(api.encode_for(vals, tc.b) if tc.enc == 0 else api.encode_dict(vals, tc.b, dct))
            if tc.enc != 0:
                dicts[tc.index] = dct
            del vals
        table = serve.Table(ctx, tcols)
        qs = synth.config5_queries(64, spec, 1.0, dicts, seed_stream=11)
        for kern, kname, rx in ((serve.PER_QUERY, "per-query", r"query_scan_kernel"),
                                (serve.SHARED, "shared-decode", r"query_shared_kernel")):
            ctx.lib.scan_query_set_kernel(ctx.h, kern)
            res = table.run([(q.filters, q.sum_col) for q in qs])
            ms = timed(lambda: table.run([(q.filters, q.sum_col) for q in qs]))
            # per query: the blocks of every column it touches that no conjunct's
            # zone map excludes, plus its conjuncts' zone maps (no sharing counted)
            byt = 0
            for q, r in zip(qs, res):
                touched = {f[0] for f in q.filters} | {q.sum_col}
                byt += r["blocks_read"] * sum(128 * spec[j].b for j in touched)
                byt += 8 * (n // 1024) * len(q.filters)
            cases.append({"name": "serving query batch, %s kernel (64 queries, 16 x 2^%d rows)" % (kname, args.n_log2),
                          "kernel": rx, "launches": args.launches + 1, "warmup": 1, "algorithmic_bytes": int(byt),
                          "values": int(sum(r["blocks_read"] for r in res) * 1024), "event_ms": ms})
        ctx.lib.scan_query_set_kernel(ctx.h, serve.SHARED)
        table.close()
        del tcols
        say("serving done")
    # --- run-length scan: the zone-map workload's column displaced by 2^16 ranks
    if "rle" not in skip:
        vals = synth.config3_column(n, s=65536, device="cuda").cpu().numpy().view(np.uint32)
        rle = api.encode_rle(vals)
        del vals
        lo, hi = synth.config3_predicate(0.1)
        ms = timed(lambda: ctx.run_rle_async(rle, lo, hi, out, zone_maps=False, all_match=False))
        cases.append({"name": "run-length scan (2^%d values, s = 2^16, %d runs, zone maps off)" % (args.n_log2, rle.runs),
                      "kernel": r"rle_scan_kernel", "launches": args.launches,
                      "algorithmic_bytes": rle.runs * 6 + ((n // 1024) + 1) * 8, "values": n, "event_ms": ms})
        del rle
        say("rle done")
    # --- materializing select: mark and write passes at b = 16
    if "select" not in skip:
        b = 16
        v = synth.config2_column(synth.config2_draws(n), b)
        col = api.encode_for(v, b)
        del v
        pos = torch.empty(n, dtype=torch.int32, device="cuda")
        for sg in (0.001, 0.1, 0.5):
            hi = synth.lt_bound(sg, b)
            cnt = int(ctx.select(col, 0, hi, zone_maps=False, out=pos).numel())
            ms = timed(lambda: ctx.select(col, 0, hi, zone_maps=False, out=pos))
            cases.append({"name": "select mark pass b=16 sigma=%g" % sg, "kernel": r"select_mark_kernel<16u?>",
                          "launches": args.launches + 1, "warmup": 1, "algorithmic_bytes": n * b // 8 + n // 8 + (n // 1024) * 4,
                          "values": n, "event_ms": ms, "group": sg})
            cases.append({"name": "select write pass b=16 sigma=%g (%d positions)" % (sg, cnt),
                          "kernel": r"select_write_kernel", "launches": args.launches + 1, "warmup": 1,
                          "algorithmic_bytes": n // 8 + 4 * cnt + (n // 1024) * 4, "values": n, "event_ms": ms,
                          "group": sg})
        say("select done")
    print(json.dumps({"n": n, "cases": cases, "cal_read_bytes": CAL_READ_BYTES,
                      "cal_triad_floats": CAL_TRIAD_FLOATS}), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
