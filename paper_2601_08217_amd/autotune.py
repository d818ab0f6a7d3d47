"""Autotuner for the launch schedule of a workload shape class.

Runs the native serving loop back to back (no pacing) on the device-resident
workload for every candidate schedule -- outputs per lane R, UEs per UL
workgroup G, where the cross-group UL sum runs (fused into the convolution
launch or a separate pass) and whether snapshots are read in place or copied
into the tap rings, whether the next item is prefetched into registers and
the persistent grid size -- and records the fastest one per workload in
``tuning.json`` next to this file.  DL results are bit-identical under every
schedule; UL sums differ only in FP32 summation order.

python -m paper_2601_08217_amd.autotune --workload 5 [--tap-fmt f32] [--slots 60]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def load_table() -> dict:
    try:
        with open(TABLE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(workload_name: str) -> dict:
    """Tuned schedule for a workload, or {} (library defaults)."""
    return load_table().get(workload_name, {})


def apply(ch, entry: dict):
    if entry:
        ch.set_tuning(entry.get("outputs_per_lane", 0), entry.get("ul_group", 0), entry.get("ul_reduce", 0),
                      entry.get("dl_group", 0), entry.get("prefetch", 0), entry.get("persist", 0),
                      entry.get("graph", 0))


def measure(dw, U, entry, warm, slots):
    import torch
    ch = dw.channel(max_ues=U, budget_bytes=1 << 30)
    apply(ch, entry)
    srv = dw.server(ch, [(0, 0)] * U, warm + slots, U, copy_taps=bool(entry.get("copy_taps", 0)))
    srv.run(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.run(slots)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    srv.close()
    ch.close()
    return dt / slots


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--tap-fmt", default="f32")
    ap.add_argument("--ues", type=int, default=0)
    ap.add_argument("--slots", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--R", default="2,4,8")
    ap.add_argument("--G", default="4,8,16,32,64")
    ap.add_argument("--DG", default="4,8,16,32")
    ap.add_argument("--reduce", default="1,2")
    ap.add_argument("--PF", default="1,2")
    ap.add_argument("--copy", default="0,1")
    ap.add_argument("--persist", default="-1,2,4", help="workgroups per CU of a persistent grid (-1: off)")
    ap.add_argument("--graph", default="2,1", help="1: replay the slot from a captured hipGraph, 2: direct")
    ap.add_argument("--write", action="store_true", help="update tuning.json with the best entry")
    ap.add_argument("--merge", default="", help="update tuning.json from the JSON line of an earlier run")
    args = ap.parse_args()
    if args.merge:
        with open(args.merge) as f:
            rec = json.loads([ln for ln in f if ln.startswith("{")][-1])
        table = load_table()
        table[rec["workload"]] = rec["best"]
        with open(TABLE, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        print(json.dumps(table[rec["workload"]]))
        return
    from . import serving as S
    from . import workload as W

    w = W.workload(args.workload, tap_fmt=args.tap_fmt, n_ues=args.ues or None)
    U = len(w.ues)
    dw = S.DeviceWorkload(w, U, x_slots=4)
    results = []
    grid = itertools.product([int(v) for v in args.R.split(",")], [int(v) for v in args.G.split(",")],
                             [int(v) for v in args.DG.split(",")], [int(v) for v in args.reduce.split(",")],
                             [int(v) for v in args.copy.split(",")], [int(v) for v in args.PF.split(",")],
                             [int(v) for v in args.persist.split(",")], [int(v) for v in args.graph.split(",")])
    for R, G, DG, red, cp, pf, ps, gr in grid:
        entry = dict(outputs_per_lane=R, ul_group=G, dl_group=DG, ul_reduce=red, copy_taps=cp, prefetch=pf,
                     persist=ps, graph=gr)
        try:
            t = measure(dw, U, entry, args.warmup, args.slots)
        except Exception as e:  # a schedule the shape cannot use (LDS budget)
            print(f"# {entry}: {e}", file=sys.stderr, flush=True)
            continue
        results.append((t, entry))
        print(f"# R={R} G={G} DG={DG} reduce={red} copy={cp} pf={pf} persist={ps} graph={gr}: "
              f"{t * 1e6:.1f} us/slot",
              file=sys.stderr, flush=True)
    results.sort(key=lambda r: r[0])
    best_t, best = results[0]
    best = dict(best, us_per_slot=round(best_t * 1e6, 1))
    out = {"workload": w.name, "best": best,
           "all": [dict(e, us_per_slot=round(t * 1e6, 1)) for t, e in results]}
    print(json.dumps(out), flush=True)
    if args.write:
        table = load_table()
        table[w.name] = best
        with open(TABLE, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
