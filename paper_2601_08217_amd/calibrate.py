"""Calibration runs for counters and ceilings: a copy of known size and an
FMA-throughput loop, both through the library's probe kernels.

python -m paper_2601_08217_amd.calibrate [--copy-mib 1024] [--reps 5]
Prints one JSON line with the measured copy bandwidth and FMA rate.

python -m paper_2601_08217_amd.calibrate --ceilings [--copy-mib 2048]
Sweeps the streaming probes (read only, write only, copy; grid sizes; plain
and non-temporal stores) and prints one JSON line with every measurement and
the best rate of each kind: the HBM ceilings kernels are compared with.
"""
import argparse
import json
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--fma-iters", type=int, default=4096)
    ap.add_argument("--skip-fma", action="store_true")
    ap.add_argument("--ceilings", action="store_true", help="sweep the read / write / copy probes")
    ap.add_argument("--grids", default="128,256,512,1024,2048,4096,8192,16384",
                    help="workgroups per probe launch (--ceilings)")
    args = ap.parse_args()
    import torch
    from . import binding as B
    if args.ceilings:
        print(json.dumps(ceilings(args.copy_mib << 20, [int(g) for g in args.grids.split(",")], args.reps)),
              flush=True)
        return 0

    nbytes = args.copy_mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    B.probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.reps):
        B.probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, s)
    e1.record(s)
    torch.cuda.synchronize()
    copy_s = e0.elapsed_time(e1) / 1e3 / args.reps
    out = {"copy_bytes": nbytes, "copy_us": copy_s * 1e6, "copy_gbs_rw": 2 * nbytes / copy_s / 1e9}
    if not args.skip_fma:
        blocks = 256 * 32
        o = torch.empty(blocks * 256, dtype=torch.float32, device="cuda:0")
        B.probe_fma(o.data_ptr(), blocks, 16, s)
        torch.cuda.synchronize()
        e0.record(s)
        B.probe_fma(o.data_ptr(), blocks, args.fma_iters, s)
        e1.record(s)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        flop = 2.0 * blocks * 256 * args.fma_iters * 64
        out.update(fma_tflops=flop / t / 1e12)
    print(json.dumps(out), flush=True)


def ceilings(nbytes: int, grids, reps: int) -> dict:
    """Bytes per second of each streaming probe form over `nbytes` buffers
    (bytes read plus bytes written, divided by the launch's event time)."""
    import torch
    from . import binding as B
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    sink = torch.empty(max(grids) * 4, dtype=torch.float32, device="cuda:0")
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for kind in ("read", "write", "copy"):
        for nt in ((False,) if kind == "read" else (False, True)):
            for g in grids:
                d = sink.data_ptr() if kind == "read" else dst.data_ptr()
                sp = 0 if kind == "write" else src.data_ptr()
                B.probe_stream(kind, d, sp, nbytes, g, nt, s)
                torch.cuda.synchronize()
                e0.record(s)
                for _ in range(reps):
                    B.probe_stream(kind, d, sp, nbytes, g, nt, s)
                e1.record(s)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) / 1e3 / reps
                moved = nbytes * (2 if kind == "copy" else 1)
                rows.append(dict(kind=kind, nontemporal=nt, blocks=g, us=round(t * 1e6, 1),
                                 gbs=round(moved / t / 1e9, 1)))
    best = {k: max((r for r in rows if r["kind"] == k), key=lambda r: r["gbs"]) for k in ("read", "write", "copy")}
    # scattered 8 KiB output chunks (the convolution's store pattern), by the
    # number of regions written at once
    chunked = []
    for streams in (1, 16, 80, 320, 1024):
        for nt in (False, True):
            for g in (256, 2048, 16384):
                B.probe_chunked_write(dst.data_ptr(), nbytes, streams, g, nt, s)
                torch.cuda.synchronize()
                e0.record(s)
                for _ in range(reps):
                    B.probe_chunked_write(dst.data_ptr(), nbytes, streams, g, nt, s)
                e1.record(s)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) / 1e3 / reps
                moved = (nbytes // 8192 // streams) * streams * 8192
                chunked.append(dict(streams=streams, nontemporal=nt, blocks=g, us=round(t * 1e6, 1),
                                    gbs=round(moved / t / 1e9, 1)))
    return dict(bytes=nbytes, reps=reps, best=best, rows=rows, chunked_write=chunked)


if __name__ == "__main__":
    sys.exit(main())
