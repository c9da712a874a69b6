"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2605_19796_amd.profiling kernel-stats DIR OUT.txt --command "..." [--top N]
    python -m paper_2605_19796_amd.profiling traffic --kernel NAME --fetch DIR --write DIR \\
        --calib-fetch DIR --calib-write DIR --out OUT.json --commands "..." "..."
    python -m paper_2605_19796_amd.profiling traffic-per-call --kernel NAME [NAME ...] \\
        --calls C --points P --workload "..." --fetch DIR --write DIR --calib-fetch DIR \\
        --calib-write DIR --out OUT.json --commands "..." "..."

    python -m paper_2605_19796_amd.profiling sq-counters DIR [DIR ...] --kernel NAME [NAME ...] \
        --points P --out OUT.txt --commands "..." "..."

kernel-stats: the per-kernel table of a `rocprofv3 --kernel-trace --stats` run (calls, total
and average duration), as text: the N kernels of largest total time (default 15).

traffic: HBM bytes per launch of one kernel from two `rocprofv3 --pmc` runs (FETCH_SIZE, then
WRITE_SIZE), each scaled by what the same counter reports for a plain device copy of known
size (bench.py --copy-calibration), so that the figure does not depend on the counter's unit.
The summary records the hash of the kernel sources it was taken on; bench.py reports the
traffic only while that hash matches.

sq-counters: per-dispatch averages of the shader-sequencer counters of the named kernels (one
`--pmc` run per directory), with instructions per grid point (wave instructions, that is
per 64 lanes) and the shares of the summed wave lifetime (SQ_WAVE_CYCLES) spent issuing VALU
and LDS instructions, waiting, and in LDS bank conflicts.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _one(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def kernel_stats(d, out, command, top=15):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_stats.csv")))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "#",
             f"{'calls':>7} {'total_ms':>10} {'avg_us':>10} {'pct':>6}  kernel"]
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}  "
                     f"{r['Name'][:150]}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(d, counter, match):
    """Per-dispatch values of `counter` for kernels whose name contains `match`."""
    vals = []
    for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
        if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {match!r} in {d}")
    return vals


def _largest(d, counter):
    vals = []
    for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
        if r["Counter_Name"] == counter:
            vals.append((float(r["Counter_Value"]), r["Kernel_Name"]))
    return max(vals)


def traffic(args):
    sys.path.insert(0, ROOT)
    import bench
    fetch = _counter(args.fetch, "FETCH_SIZE", args.kernel)
    write = _counter(args.write, "WRITE_SIZE", args.kernel)
    cf, cf_name = _largest(args.calib_fetch, "FETCH_SIZE")
    cw, cw_name = _largest(args.calib_write, "WRITE_SIZE")
    kf = bench.COPY_BYTES / cf  # bytes per counter unit
    kw = bench.COPY_BYTES / cw
    f_avg = sum(fetch) / len(fetch)
    w_avg = sum(write) / len(write)
    res = {
        "kernel": args.kernel,
        "workload": "512^3 four-width box filter step (bench.py --profile-run); algorithmic bytes "
                    "per launch: the step's 176 B per point spread over its four launches",
        "kernel_source_sha256_16": bench.kernel_source_hash(),
        "fetch_counter_avg": f_avg, "write_counter_avg": w_avg,
        "dispatches": [len(fetch), len(write)],
        "copy_calibration": {"bytes": bench.COPY_BYTES, "fetch_counter": cf, "write_counter": cw,
                             "fetch_kernel": cf_name[:80], "write_kernel": cw_name[:80],
                             "bytes_per_fetch_unit": kf, "bytes_per_write_unit": kw},
        "fetch_bytes_per_launch": f_avg * kf,
        "write_bytes_per_launch": w_avg * kw,
        "bytes_per_launch": f_avg * kf + w_avg * kw,
        "algorithmic_bytes_per_launch": bench.BYTES_PER_LAUNCH * 512 ** 3,
        "commands": args.commands,
    }
    if args.rdreq and args.cal_rdreq:
        # cross-check: L2-to-fabric read requests by size (32, 64 and 128 bytes)
        def req_bytes(d, match):
            tot = 0.0
            for c, b in (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64),
                         ("TCC_EA0_RDREQ_128B_sum", 128)):
                v = _counter(d, c, match)
                tot += b * sum(v) / len(v)
            return tot
        res["read_bytes_by_request_size"] = {
            "kernel": req_bytes(args.rdreq, args.kernel),
            "copy": req_bytes(args.cal_rdreq, cf_name[:40]),
            "counters": "TCC_EA0_RDREQ_{32B,64B,128B}_sum",
        }
    json.dump(res, open(args.out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def traffic_per_call(args):
    """HBM bytes of one call of a multi-launch entry point: each kernel's FETCH_SIZE and
    WRITE_SIZE summed over its dispatches, divided by the number of calls, copy-calibrated."""
    sys.path.insert(0, ROOT)
    import bench
    cf, _ = _largest(args.calib_fetch, "FETCH_SIZE")
    cw, _ = _largest(args.calib_write, "WRITE_SIZE")
    kf, kw = bench.COPY_BYTES / cf, bench.COPY_BYTES / cw
    res = {"workload": args.workload, "calls": args.calls, "points": args.points,
           "bytes_per_fetch_unit": kf, "bytes_per_write_unit": kw, "kernels": {},
           "commands": args.commands}
    for k in args.kernel:
        f = _counter(args.fetch, "FETCH_SIZE", k)
        w = _counter(args.write, "WRITE_SIZE", k)
        fb, wb = sum(f) * kf / args.calls, sum(w) * kw / args.calls
        res["kernels"][k] = {"dispatches": len(f), "fetch_bytes_per_call": fb,
                             "write_bytes_per_call": wb,
                             "bytes_per_point": (fb + wb) / args.points}
    json.dump(res, open(args.out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def sq_counters(args):
    vals = {k: {} for k in args.kernel}
    for d in args.dirs:
        for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
            for k in args.kernel:
                if k in r["Kernel_Name"]:
                    vals[k].setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = ["# rocprofv3 SQ counters, per-dispatch averages", "# commands:"]
    lines += [f"#   {c}" for c in args.commands]
    lines.append(f"# per point: divided by {args.points:.6g} grid points; shares: of SQ_WAVE_CYCLES")
    for k in args.kernel:
        a = {c: sum(v) / len(v) for c, v in vals[k].items()}
        if not a:
            raise SystemExit(f"no counter rows for {k!r}")
        lines.append(f"{k}:")
        for c in sorted(a):
            per = f"  ({a[c] / args.points:.3f} per point)" if c.startswith("SQ_INSTS") else ""
            lines.append(f"  {c:24s} {a[c]:16.6g}{per}")
        wc = a.get("SQ_WAVE_CYCLES")
        if wc:
            for c in ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT",
                      "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY"):
                if c in a:
                    lines.append(f"  share {c:18s} {a[c] / wc:8.3f}")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernel-stats")
    a.add_argument("dir")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--top", type=int, default=15)
    b = sub.add_parser("traffic")
    for k in ("kernel", "fetch", "write", "calib_fetch", "calib_write", "out"):
        b.add_argument("--" + k.replace("_", "-"), required=True, dest=k)
    b.add_argument("--commands", nargs="+", required=True)
    b.add_argument("--rdreq", default=None, help="run with the read-request size counters")
    b.add_argument("--cal-rdreq", default=None, dest="cal_rdreq")
    c = sub.add_parser("traffic-per-call")
    for k in ("fetch", "write", "calib_fetch", "calib_write", "out", "workload"):
        c.add_argument("--" + k.replace("_", "-"), required=True, dest=k)
    c.add_argument("--kernel", nargs="+", required=True)
    c.add_argument("--calls", type=int, required=True)
    c.add_argument("--points", type=float, required=True)
    c.add_argument("--commands", nargs="+", required=True)
    e = sub.add_parser("sq-counters")
    e.add_argument("dirs", nargs="+")
    e.add_argument("--kernel", nargs="+", required=True)
    e.add_argument("--points", type=float, required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--commands", nargs="+", required=True)
    args = ap.parse_args()
    if args.cmd == "sq-counters":
        sq_counters(args)
    elif args.cmd == "kernel-stats":
        kernel_stats(args.dir, args.out, args.command, args.top)
    elif args.cmd == "traffic":
        traffic(args)
    else:
        traffic_per_call(args)


if __name__ == "__main__":
    main()
