"""Summarise rocprofv3 CSV output of profile_run.py into a short text report
and the HBM-traffic table bench.py reads.

    python -m paper_2606_22423_amd.profile_summary --trace DIR/x_kernel_trace.csv \\
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
    """'void scan_dev::code_scan<31, 2, 0, 0, 2, 0>(scan_dev::Params)' -> 'code_scan<B=31,li/bf/nozm>'
    (either step depth: the timed region runs the one the autotuner chose)."""
    m = re.search(r"code_scan<(\d+), (\d+), (\d+), (\d+), (\d+)(?:, \d+)?>", name)
    if m:
        b, dec, mode = int(m.group(1)), int(m.group(2)), int(m.group(3))
        return "code_scan<B=%d,%s/%s/nozm>" % (b, DEC[dec], "sv" if mode else "bf")
    m = re.search(r"(beta_read_kernel<\d+>|beta_triad_kernel|cache_flush_kernel|delta_scan<[^>]*>)", name)
    return m.group(1) if m else name[:80]


def read_counters(path, counter, last):
    """(kernel short name -> values of its last `last` dispatches (KiB),
    calibration values: the dispatches before the first scan)."""
    rows = []
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter:
                rows.append((int(row["Dispatch_Id"]), short_name(row["Kernel_Name"]), float(row["Counter_Value"])))
    rows.sort()
    first_scan = min([d for d, k, _ in rows if k.startswith("code_scan")] or [0])
    per = defaultdict(list)
    cal = defaultdict(list)
    for d, k, v in rows:
        per[k].append(v)
        if d < first_scan:
            cal[k].append(v)
    return {k: v[-last:] for k, v in per.items()}, cal


def read_trace(path, last):
    """kernel short name -> durations (ns) of its last `last` dispatches."""
    rows = []
    with open(path) as fh:
        for row in csv.DictReader(fh):
            rows.append((int(row["Dispatch_Id"]), short_name(row["Kernel_Name"]),
                         int(row["End_Timestamp"]) - int(row["Start_Timestamp"])))
    rows.sort()
    per = defaultdict(list)
    for _, k, t in rows:
        per[k].append(t)
    return {k: v[-last:] for k, v in per.items()}


SELECT_STEPS = ("select_setup_kernel", "select_mark_kernel", "scan_tiles_kernel", "scan_top_kernel",
                "scan_add_kernel", "select_write_kernel", "__amd_rocclr_copyBuffer")


def select_section(trace_path, bench_line, command):
    """Per-kernel durations of the bench's materializing-select leg: each
    (b, sigma) row of the bench line is one warm-up call and three timed calls,
    each call a run of SELECT_STEPS starting at its setup kernel; the table
    averages the timed calls."""
    rows = []
    with open(trace_path) as fh:
        for row in csv.DictReader(fh):
            nm = re.sub(r"\(.*", "", row["Kernel_Name"]).replace("void ", "").replace("scan_dev::", "")
            nm = re.sub(r"<.*>", "", nm)
            if nm in SELECT_STEPS:
                rows.append((int(row["Dispatch_Id"]), nm, int(row["End_Timestamp"]) - int(row["Start_Timestamp"]),
                             int(row["Start_Timestamp"]), int(row["End_Timestamp"])))
    rows.sort()
    # A call runs from its setup kernel through the first copy after its
    # write pass (the count back to the host); copies dispatched later by
    # other parts of the program do not belong to it.
    calls, cur, closed = [], None, True
    for d, nm, t, s0, s1 in rows:
        if nm == "select_setup_kernel":
            cur, closed = [], False
            calls.append(cur)
        if cur is None or closed:
            continue
        cur.append((nm, t, s0, s1))
        if nm == "__amd_rocclr_copyBuffer" and any(k == "select_write_kernel" for k, _, _, _ in cur):
            closed = True
    sel = bench_line["select"]
    lines = ["# rocprofv3 summary: materializing select on one MI355X", "", "Commands (repository root):", ""]
    lines += ["    " + c for c in command.split(" ;; ")]
    n = bench_line["config"]["values_per_step"] // 32
    lines += ["", "Workload: the bench's select leg on its resident columns (2^%d frame-of-reference values per "
              "width, uniform in [0, 2^b), predicate v < round(sigma * 2^b), zone maps off, an output buffer of "
              "n entries so that one call runs every pass with one wait).  Per row: the mean over the three "
              "timed calls of each kernel's duration (us) and of the call's span from the first kernel's start "
              "to the last one's end; the bench's own figure (HIP events around the call) beside it."
              % (n.bit_length() - 1), ""]
    hdr = ["b", "sigma", "selected"] + [k.replace("_kernel", "").replace("__amd_rocclr_copyBuffer", "copy total")
                                        for k in SELECT_STEPS] + ["span us", "bench ms"]
    lines += ["| " + " | ".join(hdr) + " |", "|" + "---|" * len(hdr)]
    if len(calls) < 4 * len(sel):
        lines.append("(trace holds %d select calls, expected %d)" % (len(calls), 4 * len(sel)))
        return lines
    calls = calls[-4 * len(sel):]
    for i, r in enumerate(sel):
        timed = calls[4 * i + 1: 4 * i + 4]
        avg = {}
        for k in SELECT_STEPS:
            v = [t for c in timed for nm, t, _, _ in c if nm == k]
            avg[k] = sum(v) / len(v) / 1e3 if v else 0.0
        span = sum((max(e for _, _, _, e in c) - c[0][2]) for c in timed) / len(timed) / 1e3
        lines.append("| %d | %g | %d | %s | %.1f | %.4f |" % (
            r["b"], r["sigma"], r["selected"], " | ".join("%.1f" % avg[k] for k in SELECT_STEPS), span, r["ms"]))
    return lines


def _dispatches(path, counter=None):
    """[(dispatch id, raw kernel name, value)] of a kernel trace (value: the
    duration in ns) or of one counter of a counter-collection CSV."""
    rows = []
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if counter is None:
                rows.append((int(row["Dispatch_Id"]), row["Kernel_Name"],
                             int(row["End_Timestamp"]) - int(row["Start_Timestamp"])))
            elif row["Counter_Name"] == counter:
                rows.append((int(row["Dispatch_Id"]), row["Kernel_Name"], float(row["Counter_Value"])))
    rows.sort()
    return rows


def _assign(cases, rows):
    """Per case, the values of its dispatches: cases run in order, so each
    takes the next `launches` dispatches whose name matches its regular
    expression (the first of a case with a warm-up launch is dropped by the
    caller through `launches`)."""
    cursor = {}
    out = []
    for c in cases:
        rx = re.compile(c["kernel"])
        pos = cursor.get(c["kernel"], 0)
        got = []
        while pos < len(rows) and len(got) < c["launches"]:
            if rx.search(rows[pos][1]):
                got.append(rows[pos][2])
            pos += 1
        cursor[c["kernel"]] = pos
        out.append(got)
    return out


def _med(v):
    v = sorted(v)
    return v[len(v) // 2] if v else None


def paths_summary(run, trace, fetch, write, sq, command):
    """Markdown table of the profile_paths.py cases (trace, HBM bytes, SQ counters)."""
    cases = run["cases"]
    dur = _assign(cases, _dispatches(trace))
    lines = ["# rocprofv3 summary: dictionary, delta, batch, serving, run-length and select kernels on one MI355X",
             "", "Commands (repository root):", ""]
    lines += ["    " + c for c in command.split(" ;; ")]
    lines += ["", "Workload (`paper_2606_22423_amd/profile_paths.py`): 2^%d-value columns (the sweep's length) for the "
              "dictionary (2^b sorted int64 entries, 10 %% of the codes selected), delta (cumulative sums of b-bit "
              "draws, 10 %% selected) and select (b = 16) cases, the 4096-column mixed workload for the batch class "
              "kernels (default strategy: row-major direct, branch-free, zone maps), a 64-query batch on the 16-column "
              "serving table, and the zone-map workload's column displaced by 2^16 ranks, run-length encoded.  Cold "
              "cache before every launch (512 MiB read of scratch).  Algorithmic bytes: the payload bytes of the "
              "blocks the kernel must decode (after zone maps where used), plus zone maps, bases, dictionaries, "
              "ballots and positions as each kernel's notes say; GB/s and the fraction of the 8 TB/s peak are on the "
              "kernel-trace duration." % (run["n"].bit_length() - 1), ""]
    lines += ["| case | launches | avg us | algorithmic bytes | algorithmic GB/s | fraction of 8 TB/s |",
              "|---|---|---|---|---|---|"]
    for c, d in zip(cases, dur):
        d = d[c.get("warmup", 0):]  # a case's first launch may be an untimed warm-up
        if not d:
            lines.append("| %s | 0 | - | %d | - | - |" % (c["name"], c["algorithmic_bytes"]))
            continue
        avg = sum(d) / len(d)
        lines.append("| %s | %d | %.1f | %d | %.0f | %.3f |" % (c["name"], len(d), avg / 1e3, c["algorithmic_bytes"],
                                                                c["algorithmic_bytes"] / avg,
                                                                c["algorithmic_bytes"] / avg / 8000.0))
    if fetch and write:
        frows, wrows = _dispatches(fetch, "FETCH_SIZE"), _dispatches(write, "WRITE_SIZE")
        f_cal = sorted(v for _, k, v in frows if "beta_read" in k)
        w_cal = sorted(v for _, k, v in wrows if "beta_triad" in k)
        sf = _med(f_cal) * 1024 / run["cal_read_bytes"] if f_cal else None
        sw = _med(w_cal) * 1024 / (run["cal_triad_floats"] * 4) if w_cal else None
        fv, wv = _assign(cases, frows), _assign(cases, wrows)
        lines += ["", "HBM traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch, medians over the case's launches), each "
                  "scaled by the same counter's reading for a kernel of known traffic run first (FETCH factor %.4f: "
                  "streaming read of %d bytes; WRITE factor %.4f: triad, 4 B written per float)."
                  % (sf or 0, run["cal_read_bytes"], sw or 0), "",
                  "| case | FETCH KiB | WRITE KiB | scaled bytes | algorithmic bytes | ratio |", "|---|---|---|---|---|---|"]
        for c, f, w in zip(cases, fv, wv):
            fm, wm = _med(f), _med(w)
            if fm is None or wm is None or not sf or not sw:
                continue
            tb = fm * 1024 / sf + wm * 1024 / sw
            lines.append("| %s | %.0f | %.1f | %.0f | %d | %.3f |" % (c["name"], fm, wm, tb, c["algorithmic_bytes"],
                                                                       tb / c["algorithmic_bytes"]))
    if sq:
        names = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT",
                 "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "SQ_INSTS_VMEM")
        got = {nm: _assign(cases, _dispatches(sq, nm)) for nm in names}
        lines += ["", "SQ counters (medians over the case's launches; instruction counts are per wavefront, shown per "
                  "decoded value as count x 64 / values): VALU, SALU, LDS and vector-memory instructions per value, "
                  "LDS bank-conflict cycles per LDS instruction, and the share of wavefront cycles with a VALU "
                  "instruction issued.", "",
                  "| case | waves | VALU / value | SALU / value | LDS / value | VMEM / value | bank-conflict cycles / LDS instr. | VALU-active cycles |",
                  "|---|---|---|---|---|---|---|---|"]
        for i, c in enumerate(cases):
            v = {nm: _med(got[nm][i]) for nm in names}
            if v["SQ_INSTS_VALU"] is None or not c.get("values"):
                continue
            nv = c["values"]
            lines.append("| %s | %d | %.2f | %.2f | %.3f | %.3f | %s | %s |" % (
                c["name"], v["SQ_WAVES"] or 0, v["SQ_INSTS_VALU"] * 64 / nv, (v["SQ_INSTS_SALU"] or 0) * 64 / nv,
                (v["SQ_INSTS_LDS"] or 0) * 64 / nv, (v["SQ_INSTS_VMEM"] or 0) * 64 / nv,
                "%.2f" % (v["SQ_LDS_BANK_CONFLICT"] / v["SQ_INSTS_LDS"]) if v["SQ_LDS_BANK_CONFLICT"] is not None and
                v["SQ_INSTS_LDS"] else "-",
                "%.3f" % (v["SQ_ACTIVE_INST_VALU"] / v["SQ_WAVE_CYCLES"]) if v["SQ_WAVE_CYCLES"] else "-"))
    return lines


def load_bench_record(path):
    """The full bench record: bench.py's detail file (its "line" object), or
    an older stdout holding the whole record as its last JSON line."""
    with open(path) as fh:
        text = fh.read()
    try:
        d = json.loads(text)
        return d["line"] if "line" in d else d
    except ValueError:
        return json.loads([ln for ln in text.splitlines() if ln.startswith("{")][-1])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True, help="kernel_trace.csv of the --kernel-trace run")
    ap.add_argument("--last", type=int, default=5, help="timed launches per kernel (after autotuning)")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--run-json", help="stdout of profile_run.py")
    ap.add_argument("--bench-json", help="stdout of a bench.py run (its dominant kernel and timed launches)")
    ap.add_argument("--command", required=True, help="the commands that produced the CSVs")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic-json")
    ap.add_argument("--sq", help="counter_collection.csv of an SQ_* pass")
    ap.add_argument("--select-out", help="with --bench-json: also write the select leg's kernel table here")
    ap.add_argument("--paths-json", help="stdout of profile_paths.py: summarise its cases instead")
    args = ap.parse_args(argv)

    if args.paths_json:
        with open(args.paths_json) as fh:
            run = json.loads([ln for ln in fh if ln.startswith("{")][-1])
        lines = paths_summary(run, args.trace, args.fetch, args.write, args.sq, args.command)
        with open(args.out, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return 0

    if args.bench_json:
        line = load_bench_record(args.bench_json)
        rf = line["roofline"]
        m = re.match(r"code_scan<B=(\d+),([a-z_]+)/([a-z]+)/nozm>", rf["kernel"])
        run = {"n": line["config"]["values_per_step"] // 32,
               "pairs": [{"b": int(m.group(1)), "strategy": "%s/%s" % (m.group(2), m.group(3)), "tune": None,
                          "algorithmic_bytes": rf["algorithmic_bytes_per_launch"]}],
               "cal_read_bytes": line["beta_buffer_bytes"], "cal_triad_floats": line["triad_floats"],
               "bench_avg_launch_ms": rf["avg_launch_ms"],
               "timed_kernels": ["code_scan<B=%d,%s>" % (r["b"], r["strategy"]) for r in line["per_b"]]}
        args.last = line["steps"]
    else:
        with open(args.run_json) as fh:
            run = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    trace = read_trace(args.trace, args.last)
    lines = ["# rocprofv3 summary: scan kernels on one MI355X", "", "Commands (repository root):", ""]
    lines += ["    " + c for c in args.command.split(" ;; ")]
    if args.bench_json:
        lines += ["", "Workload: the bench's timed region (32 FOR columns of 2^%d uniform values, one per width, "
                  "v < round(0.1 * 2^b), zone maps off, each column read once per step).  The rows are the dominant "
                  "kernel's last %d dispatches, i.e. the timed steps; bench.py measured %.4f ms per launch with HIP "
                  "events in the same run." % (run["n"].bit_length() - 1, args.last, run["bench_avg_launch_ms"]), ""]
    else:
        lines += ["", "Workload: FOR columns of 2^%d uniform values, predicate v < round(0.1 * 2^b), zone maps off, "
                  "cold cache per launch (512 MiB read of scratch between launches); each (width, strategy) pair autotuned "
                  "as in bench.py, then launched %d times; the rows below are those %d launches (kernel trace)."
                  % (run["n"].bit_length() - 1, args.last, args.last), ""]
    lines += [
              "| kernel | launch shape (threads, WGs/CU, window) | avg us | min us | max us | algorithmic bytes | "
              "algorithmic GB/s (avg) | fraction of 8 TB/s |", "|---|---|---|---|---|---|---|---|"]
    algo, shape = {}, {}
    for p in run["pairs"]:
        key = "code_scan<B=%d,%s/nozm>" % (p["b"], p["strategy"])
        algo[key] = p["algorithmic_bytes"]
        shape[key] = p.get("tune")
    for k in sorted(algo, key=lambda k: -algo[k]):
        ts = trace.get(k, [])
        if not ts:
            continue
        avg = sum(ts) / len(ts)
        lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %d | %.0f | %.3f |" % (
            k, shape[k], avg / 1e3, min(ts) / 1e3, max(ts) / 1e3, algo[k], algo[k] / avg, algo[k] / avg / 8000.0))
    traffic = {}
    if args.fetch and args.write:
        fetch, fcal = read_counters(args.fetch, "FETCH_SIZE", args.last)
        write, wcal = read_counters(args.write, "WRITE_SIZE", args.last)
        cal_r = run["cal_read_bytes"]
        cal_w = run["cal_triad_floats"] * 4
        f_cal = sorted(v for k, vs in fcal.items() if k.startswith("beta_read") for v in vs)
        w_cal = sorted(wcal.get("beta_triad_kernel", []))
        sf = f_cal[len(f_cal) // 2] * 1024 / cal_r if f_cal else None
        sw = w_cal[len(w_cal) // 2] * 1024 / cal_w if w_cal else None
        lines += ["", "HBM traffic from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled by the counter's",
                  "reading for a kernel of known traffic dispatched before any scan: FETCH factor %.4f "
                  "(streaming read of %d bytes), WRITE factor %.4f (triad, 4 B written per float)."
                  % (sf or 0, cal_r, sw or 0), "",
                  "| kernel | FETCH KiB (median) | WRITE KiB (median) | scaled bytes per launch | algorithmic bytes | ratio |",
                  "|---|---|---|---|---|---|"]
        keys = sorted(algo)
        extra = []
        if args.bench_json:
            # every per-width scan kernel of the bench's timed region (shown),
            # and every other strategy its sweep ran on the same columns (kept
            # in the traffic table only): algorithmic bytes n * b / 8
            for k in run["timed_kernels"]:
                if k in fetch and k in write and k not in algo:
                    algo[k] = run["n"] * int(re.match(r"code_scan<B=(\d+),", k).group(1)) // 8
                    keys.append(k)
            for k in sorted(fetch):
                m = re.match(r"code_scan<B=(\d+),[a-z_]+/[a-z]+/nozm>", k)
                if m and k in write and k not in algo:
                    algo[k] = run["n"] * int(m.group(1)) // 8
                    extra.append(k)
            keys.sort(key=lambda k: -algo[k])
        for k in keys:
            fv, wv = sorted(fetch.get(k, [])), sorted(write.get(k, []))
            if not fv or not wv or not sf or not sw:
                continue
            fm, wm = fv[len(fv) // 2], wv[len(wv) // 2]
            tb = fm * 1024 / sf + wm * 1024 / sw
            traffic[k] = {"bytes_per_launch": int(tb), "fetch_kib": fm, "write_kib": wm}
            lines.append("| `%s` | %.0f | %.1f | %.0f | %d | %.3f |" % (k, fm, wm, tb, algo[k], tb / algo[k]))
        ratios = []
        for k in extra:
            fv, wv = sorted(fetch[k]), sorted(write[k])
            if not fv or not wv or not sf or not sw:
                continue
            fm, wm = fv[len(fv) // 2], wv[len(wv) // 2]
            tb = fm * 1024 / sf + wm * 1024 / sw
            traffic[k] = {"bytes_per_launch": int(tb), "fetch_kib": fm, "write_kib": wm}
            ratios.append(tb / algo[k])
        if ratios:
            lines += ["", "The sweep's other %d (width, strategy) kernels on the same columns (in the traffic table, "
                      "not shown): scaled bytes / algorithmic bytes between %.3f and %.3f."
                      % (len(ratios), min(ratios), max(ratios))]
    if args.sq:
        names = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM", "SQ_ACTIVE_INST_VALU",
                 "SQ_WAVE_CYCLES")
        sq = {nm: read_counters(args.sq, nm, args.last)[0] for nm in names}
        lines += ["", "SQ counters (medians of the same launches; instructions are per wavefront, shown per value",
                  "as count x 64 / values): VALU, SALU, LDS and vector-memory instructions per value, and the",
                  "share of wavefront cycles with a VALU instruction issued.", "",
                  "| kernel | waves | VALU / value | SALU / value | LDS / value | VMEM / value | VALU-active cycles |",
                  "|---|---|---|---|---|---|---|"]
        for k in sorted(algo, key=lambda k: -algo[k]):
            vals = {}
            for nm in names:
                v = sorted(sq[nm].get(k, []))
                vals[nm] = v[len(v) // 2] if v else None
            if vals["SQ_INSTS_VALU"] is None:
                continue
            nv = run["n"]
            lines.append("| `%s` | %d | %.2f | %.2f | %.3f | %.3f | %.3f |" % (
                k, vals["SQ_WAVES"], vals["SQ_INSTS_VALU"] * 64 / nv, vals["SQ_INSTS_SALU"] * 64 / nv,
                vals["SQ_INSTS_LDS"] * 64 / nv, vals["SQ_INSTS_VMEM"] * 64 / nv,
                vals["SQ_ACTIVE_INST_VALU"] / vals["SQ_WAVE_CYCLES"] if vals["SQ_WAVE_CYCLES"] else 0.0))
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if args.select_out and args.bench_json:
        bl = load_bench_record(args.bench_json)
        cmd = args.command.replace(" --out profiles/scan_sweep_2p28_timed_region.md",
                                   " --select-out %s --out profiles/scan_sweep_2p28_timed_region.md" % args.select_out)
        with open(args.select_out, "w") as fh:
            fh.write("\n".join(select_section(args.trace, bl, cmd)) + "\n")
    if args.traffic_json and traffic:
        for k, ts in trace.items():
            if k in traffic and ts:
                traffic[k]["trace_avg_us"] = round(sum(ts) / len(ts) / 1e3, 2)
        with open(args.traffic_json, "w") as fh:
            json.dump({"kernel_source": kernel_source_hash(), "kernels": traffic}, fh, indent=1)
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
