"""Summarise rocprofv3 CSV output of profile_run.py into a short text report
and the HBM-traffic table bench.py reads.

    python -m paper_2606_22423_amd.profile_summary --stats DIR/x_kernel_stats.csv \\
        --fetch DIR2/x_counter_collection.csv --write DIR3/x_counter_collection.csv \\
        --run-json profile_run.json --command "..." --out summary.txt --traffic-json hbm_traffic.json

FETCH_SIZE and WRITE_SIZE are KiB per dispatch.  Each is scaled by what the
same counter reads for a calibration kernel of known traffic: a streaming
read of exactly 1 GiB (FETCH) and a triad writing 4 bytes per float (WRITE).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
DEC = {0: "rm_lds", 1: "rm_direct", 2: "li", 3: "bytes"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("scan_kernels.h", "device_common.h"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """'void scan_dev::code_scan<31, 2, 0, 0, 2>(scan_dev::Params)' -> 'code_scan<B=31,li/bf/nozm>'."""
    m = re.search(r"code_scan<(\d+), (\d+), (\d+), (\d+), (\d+)>", name)
    if m:
        b, dec, mode = int(m.group(1)), int(m.group(2)), int(m.group(3))
        return "code_scan<B=%d,%s/%s/nozm>" % (b, DEC[dec], "sv" if mode else "bf")
    m = re.search(r"(beta_read_kernel<\d+>|beta_triad_kernel|cache_flush_kernel|delta_scan<[^>]*>)", name)
    return m.group(1) if m else name[:80]


def read_counters(path, counter):
    """kernel short name -> list of per-dispatch values (KiB)."""
    out = defaultdict(list)
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter:
                out[short_name(row["Kernel_Name"])].append(float(row["Counter_Value"]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--run-json", required=True, help="stdout of profile_run.py")
    ap.add_argument("--command", required=True, help="the commands that produced the CSVs")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic-json")
    args = ap.parse_args(argv)

    with open(args.run_json) as fh:
        run = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    stats = {}
    with open(args.stats) as fh:
        for row in csv.DictReader(fh):
            stats[short_name(row["Name"])] = (int(row["Calls"]), float(row["AverageNs"]), float(row["MinNs"]),
                                              float(row["MaxNs"]))
    lines = ["# rocprofv3 summary: scan kernels on one MI355X", "", "Commands (repository root):", ""]
    lines += ["    " + c for c in args.command.split(" ;; ")]
    lines += ["", "Workload: FOR columns of 2^%d uniform values, predicate v < round(0.1 * 2^b), zone maps off, "
              "cold cache per launch; pairs autotuned as in bench.py." % (run["n"].bit_length() - 1), "",
              "| kernel | calls | avg us | min us | max us | algorithmic GB/s (avg) |", "|---|---|---|---|---|---|"]
    algo = {}
    for p in run["pairs"]:
        key = "code_scan<B=%d,%s/nozm>" % (p["b"], p["strategy"])
        algo[key] = p["algorithmic_bytes"]
    for k, (calls, avg, mn, mx) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        if not (k.startswith("code_scan") or k.startswith("beta")):
            continue
        gbs = "%.0f" % (algo[k] / avg) if k in algo else ""
        lines.append("| `%s` | %d | %.1f | %.1f | %.1f | %s |" % (k, calls, avg / 1e3, mn / 1e3, mx / 1e3, gbs))
    traffic = {}
    if args.fetch and args.write:
        fetch = read_counters(args.fetch, "FETCH_SIZE")
        write = read_counters(args.write, "WRITE_SIZE")
        cal_r = run["cal_read_bytes"]
        cal_w = run["cal_triad_floats"] * 4
        f_cal = sorted(fetch.get("beta_read_kernel<1>", []) + fetch.get("beta_read_kernel<2>", []))
        w_cal = sorted(write.get("beta_triad_kernel", []))
        sf = f_cal[len(f_cal) // 2] * 1024 / cal_r if f_cal else None
        sw = w_cal[len(w_cal) // 2] * 1024 / cal_w if w_cal else None
        lines += ["", "HBM traffic from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled by the counter's",
                  "reading for a kernel of known traffic: FETCH factor %.4f (1 GiB streaming read), "
                  "WRITE factor %.4f (triad, 4 B written per float)." % (sf or 0, sw or 0), "",
                  "| kernel | FETCH KiB (median) | WRITE KiB (median) | scaled bytes per launch | algorithmic bytes | ratio |",
                  "|---|---|---|---|---|---|"]
        for k in sorted(algo):
            fv, wv = sorted(fetch.get(k, [])), sorted(write.get(k, []))
            if not fv or not wv or not sf or not sw:
                continue
            fm, wm = fv[len(fv) // 2], wv[len(wv) // 2]
            tb = fm * 1024 / sf + wm * 1024 / sw
            traffic[k] = {"bytes_per_launch": int(tb), "fetch_kib": fm, "write_kib": wm}
            lines.append("| `%s` | %.0f | %.1f | %.0f | %d | %.3f |" % (k, fm, wm, tb, algo[k], tb / algo[k]))
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if args.traffic_json and traffic:
        with open(args.traffic_json, "w") as fh:
            json.dump({"kernel_source": kernel_source_hash(), "kernels": traffic}, fh, indent=1)
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
