"""Calibration runs for counters and ceilings: a copy of known size and an
FMA-throughput loop, both through the library's probe kernels.

python -m paper_2601_08217_amd.calibrate [--copy-mib 1024] [--reps 5]
Prints one JSON line with the measured copy bandwidth and FMA rate.
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
    args = ap.parse_args()
    import torch
    from . import binding as B

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


if __name__ == "__main__":
    sys.exit(main())
