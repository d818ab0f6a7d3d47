"""Summaries of rocprofv3 CSV output for the committed profile notes.

python -m paper_2601_08217_amd.profsum trace STATS_CSV OUT_MD --cmd "..."
    per-kernel calls / average / total duration table from a
    ``--kernel-trace --stats --output-format csv`` run.

python -m paper_2601_08217_amd.profsum traffic --fetch CSV --write CSV
       --copy-fetch CSV --copy-write CSV --copy-bytes B --kernel NAME
       --workload NAME --out-json JSON --out-md MD --cmd "..."
    HBM bytes per launch of one kernel from FETCH_SIZE and WRITE_SIZE runs
    (KiB per dispatch), each scaled by what the same counter reads for a copy
    kernel that moves a known number of bytes.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import statistics

KERNEL_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "tt_kernels.hip")


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def short(name: str) -> str:
    n = name.split("(")[0]
    return n.replace("void ", "")


def col(row: dict, *names):
    """Value of the first column present (rocprofv3 versions spell them differently)."""
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def trace(args):
    rows = [dict(Name=col(r, "Name", "KernelName"), Calls=col(r, "Calls"),
                 TotalDurationNs=col(r, "TotalDurationNs", "Duration (Nsec)"),
                 AverageNs=col(r, "AverageNs", "Average (Nsec)"), MinNs=col(r, "MinNs", "Min (Nsec)"),
                 MaxNs=col(r, "MaxNs", "Max (Nsec)")) for r in csv.DictReader(open(args.stats))]
    lines = [f"# Kernel trace: {args.title}", "", f"Command: `{args.cmd}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | total (ms) |", "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} |")
    if args.window:
        # the bench's timed launches: the first `skip` dispatches of the kernel
        # are the warm-up, the next `take` the timed region
        name, skip, take = args.window.rsplit(":", 2)
        skip, take = int(skip), int(take)
        per = os.path.join(os.path.dirname(args.stats),
                           os.path.basename(args.stats).replace("kernel_stats", "kernel_trace"))
        ds = sorted((int(col(r, "Start_Timestamp")), int(col(r, "End_Timestamp")))
                    for r in csv.DictReader(open(per)) if name in col(r, "Kernel_Name"))
        win = [(e - b) / 1e3 for b, e in ds[skip:skip + take]]
        if win:
            lines += ["", f"`{name}` dispatches {skip + 1}-{skip + len(win)} in start order (the timed region, after "
                          f"{skip} warm-up dispatches): average {statistics.mean(win):.2f} us, "
                          f"min {min(win):.2f}, max {max(win):.2f} (from the per-dispatch trace)."]
    if args.bench_json:
        # the JSON line bench.py printed inside the same profiled run: its HIP-event launch average
        with open(args.bench_json) as f:
            rec = json.loads([ln for ln in f if ln.startswith("{")][-1])
        rf = rec["roofline"]
        lines += ["", f"HIP-event average of `{rf['kernel']}` printed by bench.py in the same run: "
                      f"{rf['launch_us']:.2f} us per launch ({rf['achieved']} {rf['unit']}, frac {rf['frac']})."]
    lines += ["", f"Kernel source sha256[:16] at the time of the run: `{kernel_sha()}`", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def counter_per_dispatch(path: str, counter: str, kernel_sub: str):
    vals = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if col(r, "Counter_Name", "Counter-Name") != counter or kernel_sub not in col(r, "Kernel_Name", "Kernel-Name"):
            continue
        vals[col(r, "Dispatch_Id", "Dispatch-Id")] += float(col(r, "Counter_Value", "Counter-Value"))
    return list(vals.values())


def traffic(args):
    f = counter_per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    w = counter_per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    cf = counter_per_dispatch(args.copy_fetch, "FETCH_SIZE", "k_copy")
    cw = counter_per_dispatch(args.copy_write, "WRITE_SIZE", "k_copy")
    # the largest copy dispatches are the calibration copies of known size
    cf_v, cw_v = max(cf), max(cw)
    fetch_scale = args.copy_bytes / (cf_v * 1024.0)
    write_scale = args.copy_bytes / (cw_v * 1024.0)
    f_med = statistics.median(f) * 1024.0 * fetch_scale
    w_med = statistics.median(w) * 1024.0 * write_scale
    out = {"kernel": args.kernel, "workload": args.workload, "kernel_sha": kernel_sha(),
           "fetch_bytes_per_launch": f_med, "write_bytes_per_launch": w_med,
           "bytes_per_launch": f_med + w_med, "fetch_scale": fetch_scale, "write_scale": write_scale,
           "dispatches": [len(f), len(w)]}
    with open(args.out_json, "w") as fo:
        json.dump(out, fo, indent=1)
    lines = [f"# HBM traffic: `{args.kernel}` on {args.workload}", "",
             f"FETCH_SIZE command: `{args.cmd_fetch}`", "", f"WRITE_SIZE command: `{args.cmd_write}`", "",
             f"Copy calibration commands: `{args.cmd_copy}` (once with FETCH_SIZE, once with WRITE_SIZE)", "",
             "| quantity | value |", "|---|---|",
             f"| copy kernel bytes moved (each way) | {args.copy_bytes} |",
             f"| copy FETCH_SIZE (KiB) | {cf_v:.0f} |", f"| copy WRITE_SIZE (KiB) | {cw_v:.0f} |",
             f"| FETCH scale (bytes per counted byte) | {fetch_scale:.4f} |",
             f"| WRITE scale (bytes per counted byte) | {write_scale:.4f} |",
             f"| kernel dispatches (fetch, write runs) | {len(f)}, {len(w)} |",
             f"| FETCH_SIZE per launch, median (KiB) | {statistics.median(f):.0f} |",
             f"| WRITE_SIZE per launch, median (KiB) | {statistics.median(w):.0f} |",
             f"| HBM read per launch, scaled (MB) | {f_med / 1e6:.2f} |",
             f"| HBM write per launch, scaled (MB) | {w_med / 1e6:.2f} |",
             f"| HBM traffic per launch (MB) | {(f_med + w_med) / 1e6:.2f} |", "",
             f"Kernel source sha256[:16]: `{kernel_sha()}`", ""]
    with open(args.out_md, "w") as fo:
        fo.write("\n".join(lines))
    print("\n".join(lines))


def counters(args):
    """Median per dispatch of every counter a --pmc run collected for one kernel."""
    names = []
    for r in csv.DictReader(open(args.csv)):
        n = col(r, "Counter_Name", "Counter-Name")
        if n not in names:
            names.append(n)
    rows = []
    for n in names:
        v = counter_per_dispatch(args.csv, n, args.kernel)
        if v:
            rows.append((n, len(v), statistics.median(v)))
    lines = [f"# Counters: `{args.kernel}` on {args.workload}", "", f"Command: `{args.cmd}`", "",
             "| counter | dispatches | median per dispatch |", "|---|---|---|"]
    lines += [f"| {n} | {d} | {m:.6g} |" for n, d, m in rows]
    if args.note:
        lines += ["", args.note]
    lines += ["", f"Kernel source sha256[:16] at the time of the run: `{kernel_sha()}`", ""]
    with open(args.out, "w") as fo:
        fo.write("\n".join(lines))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    t.add_argument("--title", default="")
    t.add_argument("--bench-json", default="", help="stdout of the profiled bench.py run")
    t.add_argument("--window", default="", help="KERNEL:SKIP:TAKE, the timed dispatches of one kernel")
    tr = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernel", "workload", "out_json", "out_md",
              "cmd_fetch", "cmd_write", "cmd_copy"):
        tr.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    tr.add_argument("--copy-bytes", type=float, required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("out")
    c.add_argument("--kernel", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--note", default="")
    args = ap.parse_args()
    if args.cmd_name == "trace":
        trace(args)
    elif args.cmd_name == "counters":
        counters(args)
    else:
        traffic(args)


if __name__ == "__main__":
    main()
