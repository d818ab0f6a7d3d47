"""Autotuner of the launch schedule.

The schedule has two parts, both kept in ``tuning.json`` next to this file:

- ``classes``: outputs per lane R per shape class of a link, keyed
  ``<mode>_l<taps bucket>_rx<receive antennas>`` (tap mode, tap count rounded
  up to 8, 16, 32 or 64, receive antennas).  A slot runs one convolution
  launch per (receive antennas, R) that has work, so UEs with uneven tap
  counts and rates each run at the R that suits their class (Sec. III-C:
  every UE's convolution runs in parallel with the others').
- ``workloads``: per workload, the knobs that shape the whole batch: UEs per
  UL and DL workgroup, lane tiles per DL work item, where the cross-group UL
  sum runs, LDS prefetch, persistent grid, graph replay and zero-copy
  snapshots.

Tuning a workload runs the native serving loop back to back on its
device-resident sources for every candidate and keeps the fastest: first the
batch knobs, then a coordinate search over the R of each class present.  DL
results are bit-identical under every schedule; UL sums differ only in FP32
summation order.

python -m paper_2601_08217_amd.autotune --workload 3 [--write]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
KNOBS = ("outputs_per_lane", "ul_group", "ul_reduce", "dl_group", "prefetch", "persist", "graph")


def load_table() -> dict:
    try:
        with open(TABLE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {"classes": {}, "workloads": {}}
    t.setdefault("classes", {})
    t.setdefault("workloads", {})
    return t


def lookup(workload_name: str) -> dict:
    """Schedule of a workload: its batch knobs (library defaults where absent)
    and the per-class outputs per lane of every tuned class."""
    t = load_table()
    entry = dict(t["workloads"].get(workload_name, {}))
    entry["outputs_by_class"] = {k: v["outputs_per_lane"] for k, v in t["classes"].items()}
    return entry


def apply(ch, entry: dict):
    if entry:
        ch.set_tuning(*(entry.get(k, 0) for k in KNOBS), outputs_by_class=entry.get("outputs_by_class"),
                      dl_subtiles=entry.get("dl_subtiles", 0))


def classes_of(w) -> list:
    from . import binding as B
    out = set()
    for u in w.ues:
        for d in ("dl", "ul"):
            n_rx = u.n_rx if d == "dl" else w.gnb_ant
            out.add(B.class_key(u.mode, u.n_taps, n_rx))
    return sorted(out)


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
    ap.add_argument("--G", default="4,8,16", help="UEs per UL workgroup")
    ap.add_argument("--DG", default="1,4,8", help="UEs per DL workgroup")
    ap.add_argument("--DS", default="1,2", help="lane tiles per DL work item")
    ap.add_argument("--reduce", default="2,1", help="2: separate UL reduction pass, 1: fused")
    ap.add_argument("--PF", default="2,1", help="2: stage after the previous item, 1: copy into LDS during it")
    ap.add_argument("--copy", default="0", help="0: zero-copy snapshots, 1: copy into the rings")
    ap.add_argument("--persist", default="-1", help="workgroups per CU of a persistent grid (-1: off)")
    ap.add_argument("--graph", default="2", help="1: replay the slot from a captured hipGraph, 2: direct")
    ap.add_argument("--R", default="1,2,4,8", help="outputs per lane tried per shape class")
    ap.add_argument("--write", action="store_true", help="update tuning.json with the best schedule")
    ap.add_argument("--merge", default="", help="update tuning.json from the JSON line of an earlier run")
    args = ap.parse_args()
    if args.merge:
        with open(args.merge) as f:
            merge(json.loads([ln for ln in f if ln.startswith("{")][-1]))
        return
    from . import serving as S
    from . import workload as W

    w = W.workload(args.workload, tap_fmt=args.tap_fmt, n_ues=args.ues or None)
    U = len(w.ues)
    dw = S.DeviceWorkload(w, U, x_slots=4)
    base = lookup(w.name)
    log = []

    def run(entry, tag):
        try:
            t = measure(dw, U, entry, args.warmup, args.slots)
        except Exception as e:  # a schedule the shape cannot use (LDS budget)
            print(f"# {tag}: {e}", file=sys.stderr, flush=True)
            return None
        log.append(dict(tag=tag, us_per_slot=round(t * 1e6, 1)))
        print(f"# {tag}: {t * 1e6:.1f} us/slot", file=sys.stderr, flush=True)
        return t

    # batch knobs, with the classes at their current schedule
    best_t, best = None, None
    ints = lambda v: [int(x) for x in v.split(",")]
    for G, DG, DS, red, cp, pf, ps, gr in itertools.product(ints(args.G), ints(args.DG), ints(args.DS),
                                                             ints(args.reduce), ints(args.copy), ints(args.PF),
                                                             ints(args.persist), ints(args.graph)):
        e = dict(base, ul_group=G, dl_group=DG, dl_subtiles=DS, ul_reduce=red, copy_taps=cp, prefetch=pf,
                 persist=ps, graph=gr)
        t = run(e, f"G={G} DG={DG} DS={DS} reduce={red} copy={cp} pf={pf} persist={ps} graph={gr}")
        if t is not None and (best_t is None or t < best_t):
            best_t, best = t, e
    # coordinate search over the outputs per lane of each class present
    byc = dict(best.get("outputs_by_class") or {})
    for key in classes_of(w):
        for R in ints(args.R):
            trial = dict(byc, **{key: R})
            t = run(dict(best, outputs_by_class=trial), f"{key} R={R}")
            if t is not None and t < best_t:
                best_t, byc = t, trial
    best = dict(best, outputs_by_class=byc)
    out = {"workload": w.name, "us_per_slot": round(best_t * 1e6, 1),
           "classes": {k: byc[k] for k in classes_of(w) if k in byc},
           "knobs": {k: best[k] for k in ("ul_group", "dl_group", "dl_subtiles", "ul_reduce", "copy_taps",
                                          "prefetch", "persist", "graph")},
           "all": log}
    print(json.dumps(out), flush=True)
    if args.write:
        merge(out)


def merge(out: dict):
    """Record a tuning run's result: its classes' outputs per lane and its
    workload's batch knobs."""
    table = load_table()
    for k, R in out["classes"].items():
        table["classes"][k] = {"outputs_per_lane": R, "tuned_on": out["workload"]}
    table["workloads"][out["workload"]] = dict(out["knobs"], us_per_slot=out["us_per_slot"])
    with open(TABLE, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
