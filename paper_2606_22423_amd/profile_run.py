"""Short, fixed workload for rocprofv3 runs of the scan kernels.

Builds frame-of-reference columns of 2^n_log2 uniform values at the given
widths (row-major and lane-interleaved), autotunes each (width, strategy)
pair exactly as bench.py does, then launches each pair `launches` times on a
cold cache (a 512 MiB read of scratch between launches).  For the HBM byte
counters it also runs two calibration kernels of known traffic: a streaming
read of exactly 1 GiB (beta_read) and a triad over 2^26 floats (8 bytes read
and 4 written per float).

    rocprofv3 --kernel-trace --stats -- python3 -m paper_2606_22423_amd.profile_run
    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2606_22423_amd.profile_run
"""
from __future__ import annotations

import argparse
import json
import sys

CAL_READ_BYTES = 1 << 30
CAL_TRIAD_FLOATS = 1 << 26


def parse_pairs(text):
    """'31:li/bf,32:rm_lds/bf' -> [(31, 'li/bf'), (32, 'rm_lds/bf')]"""
    out = []
    for part in text.split(","):
        b, s = part.split(":")
        out.append((int(b), s))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", default="31:li/bf,32:rm_lds/bf,16:rm_direct/bf,8:rm_direct/bf",
                    help="width:decoder/mode pairs (zone maps off)")
    ap.add_argument("--n-log2", type=int, default=28)
    ap.add_argument("--launches", type=int, default=5)
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args(argv)

    import torch

    import synth
    from paper_2606_22423_amd import api
    from paper_2606_22423_amd._lib import DEC_BYTES, DEC_LI, DEC_RM_DIRECT, DEC_RM_LDS, LAYOUT_LI, strategy

    decs = {"rm_lds": DEC_RM_LDS, "rm_direct": DEC_RM_DIRECT, "li": DEC_LI, "bytes": DEC_BYTES}
    ctx = api.Context(0)
    # calibration kernels of known traffic
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

    n = 1 << args.n_log2
    draws = synth.config2_draws(n)
    evict = torch.empty(512 << 18, dtype=torch.int32, device="cuda")
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    report = []
    for width, name in parse_pairs(args.pairs):
        dname, mode = name.split("/")
        s = strategy(decs[dname], 1 if mode == "sv" else 0, 0)
        v = synth.config2_column(draws, width)
        col = api.encode_for(v, width, layout=LAYOUT_LI if dname == "li" else 0)
        hi = synth.lt_bound(0.1, width)
        cfg = None
        if not args.no_autotune:
            cfg, _ = ctx.autotune(col, 0, hi, s, reps=3)
        ev = []
        for _ in range(args.launches):
            ctx.cache_flush(evict, evict.numel() * 4)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.run_async(col, 0, hi, s, out)
            e1.record()
            ev.append((e0, e1))
        torch.cuda.synchronize()
        ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        report.append({"b": width, "strategy": name, "tune": cfg, "median_ms": ms[len(ms) // 2],
                       "algorithmic_bytes": n * width // 8})
        del col, v
    print(json.dumps({"n": n, "pairs": report, "cal_read_bytes": CAL_READ_BYTES,
                      "cal_triad_floats": CAL_TRIAD_FLOATS}), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
