#!/usr/bin/env python3
"""Throughput, latency and roofline of the channel-emulation path on one GPU.

Default workload: 256 concurrent SISO UEs, 32 LINEAR taps (snapshots every
128 samples), 61.44 Msps, 0.5 ms slots (30,720 samples), downlink per UE and
uplink summed at the gNB, ci16 IQ, FP32 accumulation, FP32 taps.  One step is
one slot of the whole path: tap ingest for every UE and direction, DL and UL
convolution, noise, quantisation and history update, driven by the native
serving loop with every input already resident in HBM.

Prints one JSON line: emulated UE-link samples per second (batched), plus
p50/p99 slot latency under 0.5 ms pacing, the plain per-UE-launch form, the
roofline of the convolution kernel and the FP64 CPU oracle on a sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 FLOP/clk (packed FP32 FMA)
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fir_c5_traffic.json")
C1_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fir_c1_x1024_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2601_08217_amd", "csrc", "tt_kernels.hip")
MGNB_LINK_BASE = 1 << 20          # tap-draw keys of the multi-gNB DL links, clear of the C5 link keys


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload: str, path: str = None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    try:
        with open(path or TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha() or t.get("workload") != workload:
        return None
    return t.get("bytes_per_launch")


def poisson_sessions(config, rate, mean_s, horizon_slots, slot_s, prefill):
    from paper_2601_08217_amd import workload as W
    ses = W.poisson_sessions(config, rate, mean_s, horizon_slots * slot_s, prefill=prefill)
    return [(int(t / slot_s), max(1, int(round(d / slot_s)))) for t, d in ses]


def sparse_leg(w, U, tune, stream, nsel: int, steps: int, warmup: int, dw_dense):
    """Sparse top-n (Sec. III-C) on the same workload: throughput, and the
    relative L2 error of its outputs against the full FIR over the same slots."""
    import numpy as np
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import serving as S

    dw = S.DeviceWorkload(w, U, x_slots=4, sparse_taps=nsel)
    forever = [(0, 0)] * U
    copy_taps = bool(tune.get("copy_taps", 0))

    def outputs(d):
        ch = d.channel(max_ues=U, budget_bytes=1 << 30, stream=stream)
        T.apply(ch, tune)
        srv = d.server(ch, forever, 2, U, copy_taps=copy_taps)
        srv.run(2)
        torch.cuda.synchronize()
        y = torch.stack([d.dl_y[j][1] for j in range(U)]).float()
        z = d.ul_z[0][1].float()
        srv.close()
        ch.close()
        return y, z

    yd, zd = outputs(dw_dense)
    ys, zs = outputs(dw)
    err_dl = float(torch.linalg.vector_norm(ys - yd) / torch.linalg.vector_norm(yd))
    err_ul = float(torch.linalg.vector_norm(zs - zd) / torch.linalg.vector_norm(zd))
    ch = dw.channel(max_ues=U, budget_bytes=1 << 30, stream=stream)
    T.apply(ch, tune)
    srv = dw.server(ch, forever, warmup + steps, U, copy_taps=copy_taps)
    srv.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    srv.close()
    ch.close()
    return dict(taps_kept=nsel, of=w.ues[0].n_taps, value=steps * w.link_samples_per_slot() / dt, unit="samples/s",
                ms_per_step=1e3 * dt / steps, rel_l2_err_vs_full_dl=round(err_dl, 5),
                rel_l2_err_vs_full_ul=round(err_ul, 5))


def ue_sweep(dw, tune, stream, counts, slots: int, warm: int = 20):
    """Paced 0.5 ms slots at increasing UE counts (sources reused cyclically,
    every UE with its own outputs): the largest count whose p99 slot latency
    stays within the slot.  All UEs join in the first warm-up slot; the paced
    window starts after the warm-up."""
    from paper_2601_08217_amd import autotune as T
    rows = []
    for n in counts:
        ch = dw.channel(max_ues=n, budget_bytes=4 << 30, stream=stream)
        T.apply(ch, tune)
        srv = dw.server(ch, [(0, 0)] * n, warm + slots, n, slot_us=500.0, copy_taps=bool(tune.get("copy_taps", 0)))
        srv.run(warm)
        srv.stats(reset=True)
        srv.run(slots)
        st = srv.stats()
        srv.close()
        ch.close()
        rows.append(dict(ues=n, lat_p50_us=round(st["lat_p50_us"], 1), lat_p99_us=round(st["lat_p99_us"], 1),
                         lat_max_us=round(st["lat_max_us"], 1), misses=st["misses"],
                         host_submit_us=round(st["host_us_mean"], 1)))
        print(f"# sweep {n} UEs: p50/p99 {st['lat_p50_us']:.0f}/{st['lat_p99_us']:.0f} us, {st['misses']} misses",
              file=sys.stderr, flush=True)
    ok = [r["ues"] for r in rows if r["lat_p99_us"] <= 500.0]
    return dict(slots_each=slots, warmup_each=warm, rows=rows, max_ues_p99_within_slot=max(ok) if ok else 0)


def pcie_leg(dw, w, U, tune, stream, slots: int):
    """Slot latency with the IQ crossing PCIe: per slot, an H2D copy from
    pinned host memory of every UE's UL input and the gNB's DL input, the
    slot, then a D2H copy of every UE's DL output and the gNB's UL output,
    serialised on the channel's stream (the copies move the slot's IQ bytes
    through a staging buffer; the kernels read the resident pools)."""
    import numpy as np
    import torch
    from paper_2601_08217_amd import autotune as T
    N = dw.cell_N[0]
    nb_in = U * N * 4 + dw.n_ant * N * 4
    nb_out = U * N * 4 + dw.n_ant * N * 4
    h_in = torch.empty(nb_in, dtype=torch.uint8, pin_memory=True)
    h_out = torch.empty(nb_out, dtype=torch.uint8, pin_memory=True)
    d_in = torch.empty(nb_in, dtype=torch.uint8, device="cuda:0")
    d_out = torch.empty(nb_out, dtype=torch.uint8, device="cuda:0")
    ch = dw.channel(max_ues=U, budget_bytes=1 << 30, stream=stream)
    T.apply(ch, tune)
    srv = dw.server(ch, [(0, 0)] * U, slots + 2, U, copy_taps=bool(tune.get("copy_taps", 0)))
    st = stream if stream is not None else torch.cuda.current_stream()
    lat = []
    for s in range(slots + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(st):
            d_in.copy_(h_in, non_blocking=True)
        srv.run(1)
        with torch.cuda.stream(st):
            h_out.copy_(d_out, non_blocking=True)
        st.synchronize()
        if s >= 2:
            lat.append(time.perf_counter() - t0)
    srv.close()
    ch.close()
    lat = np.array(lat) * 1e6
    return dict(slots=slots, bytes_h2d=nb_in, bytes_d2h=nb_out, lat_p50_us=round(float(np.percentile(lat, 50)), 1),
                lat_p99_us=round(float(np.percentile(lat, 99)), 1),
                value=float(w.link_samples_per_slot() / (lat.mean() * 1e-6)), unit="samples/s")


def trace_rate_leg(w, U, tune, stream, steps: int, period: int):
    """The C5 shape with snapshots every `period` samples (trace-like rates, the
    paper's CIR traces step every 1 ms): throughput and the convolution
    kernel's time."""
    import dataclasses
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import serving as S
    from paper_2601_08217_amd import workload as W
    ues = [dataclasses.replace(u, period=period) for u in w.ues]
    wt = dataclasses.replace(w, name=f"{w.name}_P{period}", ues=ues)
    dw = S.DeviceWorkload(wt, U, x_slots=4)
    ch = dw.channel(max_ues=U, budget_bytes=1 << 30, stream=stream)
    T.apply(ch, tune)
    srv = dw.server(ch, [(0, 0)] * U, 20 + steps, U)
    srv.run(20)
    ch.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n = ch.kernel_time(1)
    srv.close()
    ch.close()
    return dict(snapshot_period=period, value=steps * wt.link_samples_per_slot() / dt, unit="samples/s",
                us_per_slot=round(1e6 * dt / steps, 1), k_fir_us=round(ms * 1e3 / n, 1) if n else 0.0)


def trace_replay_leg(w, U, tune, stream, steps: int, n_paths: int, warmup: int = 20, step_ms: float = 1.0):
    """Trace replay (Sec. IV): every link's snapshots come from a
    continuous-delay ray trace (n_paths paths, one step per step_ms), resampled
    on the device into the tap rings between slots (LINEAR between steps);
    throughput with the resampling inside the timed loop, and the resampling
    call's own time for all links."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import binding as B
    from paper_2601_08217_amd import serving as S
    from paper_2601_08217_amd import workload as W
    u0 = w.ues[0]
    fs = u0.sample_rate
    N = w.samples_per_slot(fs)
    P = int(round(fs * step_ms * 1e-3))
    wt = dataclasses.replace(w, name=f"{w.name}_trace", ues=[dataclasses.replace(u, period=P) for u in w.ues])
    dw = S.DeviceWorkload(wt, U, x_slots=4)
    ch = dw.channel(max_ues=U, budget_bytes=1 << 30, stream=stream)
    T.apply(ch, tune)
    ids = [ch.add_ue(**dw.ue_cfg[i]) for i in range(U)]
    slots = warmup + steps
    K = slots * N // P + 6  # the loop reads steps up to (slots N - 1) // P + 1, the repeats two more
    dl_all, g_all, t0 = [], [], []
    for i in range(U):
        u = dw.shapes[i]
        for d in ("dl", "ul"):
            nrx, ntx = (u.n_rx, dw.n_ant) if d == "dl" else (dw.n_ant, u.n_tx)
            tr = W.ray_trace(w.config, W.link_key(i, d), K, nrx, ntx, n_paths, fs, step_s=step_ms * 1e-3,
                             total=1.0 if d == "dl" else W.ul_pdp_scale(w, u))
            dl_all.append(tr.delay)
            g_all.append(tr.gain.reshape(K, n_paths, -1))
            t0.append(tr.t0)
    dd = torch.from_numpy(np.stack(dl_all)).to("cuda:0")
    gd = torch.from_numpy(np.stack(g_all)).to("cuda:0")
    nrt = gd.shape[-1]
    ent = np.zeros(2 * U, B.CIR_SRC_DTYPE)
    ent["ue"] = np.repeat(ids, 2)
    ent["dir"] = np.tile([B.DIRS["dl"], B.DIRS["ul"]], U)
    ent["n_paths"] = n_paths
    ent["t0_s"] = t0
    dbase = dd.data_ptr() + np.arange(2 * U, dtype=np.uint64) * np.uint64(K * n_paths * 8)
    gbase = gd.data_ptr() + np.arange(2 * U, dtype=np.uint64) * np.uint64(K * n_paths * nrt * 8)

    def feed(k0, count):
        ent["k0"], ent["count"] = k0, count
        ent["delay_s"] = dbase + np.uint64(k0 * n_paths * 8)
        ent["gain"] = gbase + np.uint64(k0 * n_paths * nrt * 8)
        ch.set_taps_cir(ent)

    ys = [dw._zeros((2, u.n_rx, N)) for u in dw.shapes]
    prepared = [ch.prepare_slot(ids, [dw.dl_x[0][p].data_ptr()] * U, [y[p % 2].data_ptr() for y in ys], ids,
                                [x[p].data_ptr() for x in dw.ul_x], [dw.ul_z[0][p % 2].data_ptr()], [N])
                for p in range(4)]
    next_k = 0
    t_start = None
    for s in range(slots):
        if s == warmup:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        need = ((s + 1) * N - 1) // P + 1
        if need >= next_k:
            feed(next_k, need + 1 - next_k)
            next_k = need + 1
        ch.apply_prepared(prepared[s % 4])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_start
    # the resampling call alone: one step for every link, repeated
    reps = 50
    torch.cuda.synchronize()
    r0 = time.perf_counter()
    for r in range(reps):
        feed(next_k + (r % 2), 1)
    torch.cuda.synchronize()
    rs = (time.perf_counter() - r0) / reps
    ch.close()
    return dict(paths=n_paths, step_ms=step_ms, snapshot_period=P, links=2 * U, steps=steps,
                value=steps * w.link_samples_per_slot() / dt, unit="samples/s", us_per_slot=round(1e6 * dt / steps, 1),
                resample_us_per_call=round(1e6 * rs, 1))


def multi_gnb_leg(w, U, tune, stream, dw, steps: int, n_gnb: int = 3, warmup: int = 20):
    """Multi-gNB downlink (inter-cell interference, Sec. V) on the C5 shape:
    n_gnb single-antenna gNBs at the C5 rate; UE i is served by gNB i mod
    n_gnb and hears every gNB, its DL input stacking the serving gNB's stream
    first and the others in ascending order, over its own L-tap LINEAR
    Rayleigh channel per gNB (exponential PDP, C5's tap format).  The UL is
    C5's, summed at the serving gNB.  Snapshots are read in place.  Link
    samples count every (UE, gNB) DL pair and the UL."""
    import numpy as np
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import binding as B
    from paper_2601_08217_amd import serving as S
    from paper_2601_08217_amd import workload as W
    u0 = w.ues[0]
    N = w.samples_per_slot(u0.sample_rate)
    per = N // u0.period
    xs = dw.x_slots
    tl = xs * per
    served = [sum(1 for i in range(U) if i % n_gnb == g) for g in range(n_gnb)]
    offs = W.noise_offsets(w.config, 7, 4 * n_gnb, len(dw.pool16))
    cells = [dict(dw.cells[0], ul_sigma=float(W.sigma_for_snr(w.snr_db, 1.0 / max(1, served[g]))),
                  ul_noise_off=[int(v) for v in offs[4 * g:4 * g + 4]]) for g in range(n_gnb)]
    pdp = W.exp_pdp(u0.n_taps)
    dlp = []
    for i in range(U):
        h = W.rayleigh_snapshots(w.config, MGNB_LINK_BASE + i, tl, 1, n_gnb, pdp, w.tap_fmt)
        dlp.append(torch.from_numpy(np.ascontiguousarray(np.concatenate([h, h[:1]]))).to("cuda:0"))
    streams = [dw.dl_x[0]] + [
        torch.from_numpy(np.stack([W.iq_block(w.config, S.DL_STREAM_BASE + g, p, 1, N, w.iq_fmt)
                                   for p in range(xs)])).to("cuda:0") for g in range(1, n_gnb)]
    stack = [torch.cat([streams[c]] + [streams[g] for g in range(n_gnb) if g != c], dim=1).contiguous()
             for c in range(n_gnb)]
    ys = dw._zeros((U, 1, N))
    zs = dw._zeros((n_gnb, 1, N))
    ch = B.Channel(cells, U, 4 << 30, w.iq_fmt, dw.pool16, stream=stream)
    T.apply(ch, tune)
    ids = [ch.add_ue(**dict(dw.ue_cfg[i], cell=i % n_gnb, dl_tx_streams=n_gnb)) for i in range(U)]
    dsz = dlp[0][0].numel() * dlp[0].element_size()
    usz = dw.taps[0][1][0].numel() * dw.taps[0][1].element_size()
    prepared = [ch.prepare_slot(ids, [stack[i % n_gnb][p].data_ptr() for i in range(U)],
                                [ys[i].data_ptr() for i in range(U)], ids,
                                [dw.ul_x[i][p].data_ptr() for i in range(U)], [z.data_ptr() for z in zs],
                                [N] * n_gnb, dl_taps=[dlp[i].data_ptr() + p * per * dsz for i in range(U)],
                                ul_taps=[dw.taps[i][1].data_ptr() + p * per * usz for i in range(U)])
                for p in range(xs)]
    for s in range(warmup):
        ch.apply_prepared(prepared[s % xs])
    ch.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ch.apply_prepared(prepared[(warmup + s) % xs])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    fir_ms, fir_n = ch.kernel_time(1)
    ch.close()
    links = U * N * (n_gnb + 1)
    fir_us = 1e3 * fir_ms / fir_n if fir_n else 0.0
    flop = links * u0.n_taps * 12.0
    return dict(gnbs=n_gnb, ues=U, value=links / dt, unit="samples/s", us_per_slot=round(1e6 * dt, 1),
                link_samples_per_slot=links, kernels_us=dict(k_fir=round(fir_us, 1)),
                tflops_algorithmic=round(flop / dt / 1e12, 1))


def host_io_leg(w, U, tune, stream, steps: int, counts, depth: int = 3, warm: int = 10, slot_us: float = 500.0):
    """Host IQ coupling (tt_io): every slot's IQ enters from pinned host memory
    and its outputs return there, `depth` slots in flight.  Per UE count: the
    back-to-back slot rate and latency (submit to outputs in host memory),
    then the same paced at one slot per 0.5 ms as a real-time producer would
    submit.  Snapshots are fed per slot from the resident pools through
    tt_channel_set_taps_device (the zero-copy pointers of the serving loop are
    not used here)."""
    import numpy as np
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import binding as B
    from paper_2601_08217_amd import serving as S
    N = w.samples_per_slot(w.ues[0].sample_rate)
    dw = S.DeviceWorkload(w, U, x_slots=4)
    rows = []
    for n in counts:
        u0 = dw.shapes[0]
        key = lambda u: (u.n_tx, u.n_rx, u.n_taps, u.mode, u.period, u.sample_rate)
        assert all(key(dw.shapes[i]) == key(u0) for i in range(n)) and u0.mode != "jakes"
        ch = dw.channel(max_ues=n, budget_bytes=1 << 30, stream=stream)
        T.apply(ch, tune)
        ids = [ch.add_ue(**dw.ue_cfg[i]) for i in range(n)]
        io = B.HostIO(ch, 0, ids, N, depth)
        for b in range(depth):  # what a producer would have written
            v = torch.from_numpy(io.inputs(b))
            off = 0
            for t in [dw.dl_x[0][b % 4]] + [dw.ul_x[i][b % 4] for i in range(n)]:
                nb = t.numel() * t.element_size()
                v[off:off + nb].copy_(t.reshape(-1).view(torch.uint8))
                off += nb
        tl = dw.tap_len[0]
        per_bytes = dw.taps[0][0][0].numel() * dw.taps[0][0].element_size()
        ent = np.zeros(2 * n, B.TAPS_SRC_DTYPE)
        ent["ue"] = np.repeat(ids, 2)
        ent["dir"] = np.tile([B.DIRS["dl"], B.DIRS["ul"]], n)
        base = np.array([dw.taps[i][d].data_ptr() for i in range(n) for d in (0, 1)], dtype=np.uint64)
        state = dict(next_k=0)

        def feed(s):
            need = ((s + 1) * N - 1) // u0.period + 1
            k0 = state["next_k"]
            cnt = need + 1 - k0
            assert (k0 % tl) + cnt <= tl + 1
            ent["k0"], ent["count"] = k0, cnt
            ent["src"] = base + np.uint64((k0 % tl) * per_bytes)
            ch.set_taps_device(ent)
            state["next_k"] = need + 1

        def run(n_slots, pace):
            lat, late = [], 0
            busy = set()
            t0 = time.perf_counter()
            for s in range(n_slots):
                b = s % depth
                if b in busy:
                    lat.append(io.wait(b))
                    busy.discard(b)
                if pace:
                    tick = t0 + s * slot_us * 1e-6
                    while time.perf_counter() < tick:
                        io.poll()
                    late += (time.perf_counter() - tick) > slot_us * 1e-6
                feed(state["s"] + s)
                io.submit(b)
                busy.add(b)
            for b in sorted(busy, key=lambda b: (b - n_slots) % depth):
                lat.append(io.wait(b))
            dt = time.perf_counter() - t0
            state["s"] += n_slots
            return dt, np.array(lat), late

        state["s"] = 0
        run(warm, False)
        dt, lat, _ = run(steps, False)
        _, plat, late = run(steps, True)
        in_bytes, out_bytes = io.inputs(0).nbytes, io.outputs(0).nbytes
        io.close()
        ch.close()
        link = n * N * (u0.n_rx + dw.n_ant)
        rows.append(dict(ues=n, value=steps * link / dt, unit="samples/s", us_per_slot=round(1e6 * dt / steps, 1),
                         lat_p50_us=round(float(np.percentile(lat, 50)), 1),
                         lat_p99_us=round(float(np.percentile(lat, 99)), 1),
                         paced_lat_p50_us=round(float(np.percentile(plat, 50)), 1),
                         paced_lat_p99_us=round(float(np.percentile(plat, 99)), 1), paced_late_submits=int(late),
                         bytes_h2d_per_slot=int(in_bytes), bytes_d2h_per_slot=int(out_bytes)))
        print(f"# host io {n} UEs: {rows[-1]['us_per_slot']} us/slot back to back, paced p50/p99 "
              f"{rows[-1]['paced_lat_p50_us']:.0f}/{rows[-1]['paced_lat_p99_us']:.0f} us, {late} late",
              file=sys.stderr, flush=True)
    ok = [r["ues"] for r in rows if r["us_per_slot"] <= slot_us]
    return dict(depth=depth, steps_each=steps, rows=rows, max_ues_real_time=max(ok) if ok else 0)


PEAK_ALU = 157.3e12
PEAK_HBM = 8.0e12


def _roof(flop, byts, dt_slot, k_us=None, k_flop=None):
    """Both roofline fractions of one slot (algorithmic FLOP and bytes); the
    convolution kernel's ALU fraction counts its own share, k_flop."""
    k_flop = flop if k_flop is None else k_flop
    inten = flop / byts
    r = dict(flop_per_slot=flop, bytes_per_slot=byts, intensity=round(inten, 2),
             bound="alu" if inten > PEAK_ALU / PEAK_HBM else "hbm",
             slot_tflops=round(flop / dt_slot / 1e12, 2), slot_frac_alu=round(flop / dt_slot / PEAK_ALU, 3),
             slot_gbs=round(byts / dt_slot / 1e9, 1), slot_frac_hbm=round(byts / dt_slot / PEAK_HBM, 3))
    if k_us:
        r.update(k_fir_us=round(k_us, 1), k_fir_frac_alu=round(k_flop / (k_us * 1e-6) / PEAK_ALU, 3),
                 k_fir_frac_hbm=round(byts / (k_us * 1e-6) / PEAK_HBM, 3))
    return r


def _served(w, stream, slots, warm=10):
    """LINEAR workloads through the serving loop (resident pools, zero-copy snapshots)."""
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import serving as S
    U = len(w.ues)
    dw = S.DeviceWorkload(w, U, x_slots=4)
    tune = T.lookup(w.name)
    ch = dw.channel(max_ues=U, budget_bytes=4 << 30, stream=stream)
    T.apply(ch, tune)
    # the slot time untimed, then the convolution's launch time from stamped
    # launches of further slots (stamping costs small slots several us)
    timed = min(slots, 20)
    srv = dw.server(ch, [(0, 0)] * U, warm + slots + timed, U, copy_taps=bool(tune.get("copy_taps", 0)))
    srv.run(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.run(slots)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / slots
    ch.enable_kernel_timing(True)
    srv.run(timed)
    ms, n = ch.kernel_time(1)
    srv.close()
    ch.close()
    a = dw.algorithmic()
    return dict(dt=dt, k_us=ms * 1e3 / n if n else None, flop=a["flop"], fir_flop=a["fir_flop"], bytes=a["bytes"])


def _jakes_direct(w, stream, slots, warm=5, tune=None, dw=None):
    """Jakes workloads (every cell, DL and UL) with one apply_slot per slot."""
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import serving as S
    U = len(w.ues)
    dw = dw or S.DeviceWorkload(w, U, x_slots=4)
    ch = dw.channel(max_ues=U, budget_bytes=4 << 30, stream=stream)
    T.apply(ch, T.lookup(w.name) if tune is None else tune)
    ids = []
    for i in range(U):
        ids.append(ch.add_ue(**dw.ue_cfg[i]))
        for d, jp in zip(("dl", "ul"), dw.jakes[i]):
            ch.set_jakes(ids[-1], d, *jp)
    ys = [dw._zeros((2, u.n_rx, dw.cell_N[dw.rates.index(u.sample_rate)])) for u in dw.shapes]
    cell = [dw.rates.index(u.sample_rate) for u in dw.shapes]
    prepared = [ch.prepare_slot(ids, [dw.dl_x[cell[i]][p].data_ptr() for i in range(U)],
                                [ys[i][p % 2].data_ptr() for i in range(U)], ids,
                                [dw.ul_x[i][p].data_ptr() for i in range(U)],
                                [z[p % 2].data_ptr() for z in dw.ul_z], dw.cell_N) for p in range(4)]
    for s in range(warm):
        ch.apply_prepared(prepared[s % 4])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(slots):
        ch.apply_prepared(prepared[(warm + s) % 4])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / slots
    # launch times from stamped launches of further slots
    ch.enable_kernel_timing(True)
    for s in range(min(slots, 20)):
        ch.apply_prepared(prepared[(warm + slots + s) % 4])
    ms, n = ch.kernel_time(1)
    ams, an = ch.kernel_time(2)
    ch.close()
    a = dw.algorithmic()
    return dict(dt=dt, k_us=ms * 1e3 / n if n else None, flop=a["flop"], fir_flop=a["fir_flop"], bytes=a["bytes"],
                anchor_us=ams * 1e3 / an if an else None)


def _hold_dl_direct(w, n_ues, stream, calls, warm=2, tune=None):
    """C1's downlink (HOLD, cf32) for n_ues UEs sharing the gNB stream: one
    batched apply_dl per call of N samples, snapshots ingested per call."""
    import numpy as np
    import torch
    from paper_2601_08217_amd import binding as B
    from paper_2601_08217_amd import workload as W
    u0 = w.ues[0]
    N = w.samples_per_slot(u0.sample_rate)
    per_call = N // u0.period
    pool16 = W.noise_pool(w.config, 1 << 22)
    ch = B.Channel([dict(sample_rate_hz=u0.sample_rate, n_ant=1, max_samples=N)], max_ues=n_ues,
                   hbm_budget_bytes=4 << 30, iq_fmt="cf32", noise_pool=pool16, stream=stream)
    if tune:
        from paper_2601_08217_amd import autotune as T
        T.apply(ch, tune)
    ids = [ch.add_ue(cell=0, n_taps=u0.n_taps, mode="hold", snapshot_period=u0.period, ring_snapshots=1024,
                     dl_sigma=0.1, dl_noise_off=[97 * u]) for u in range(n_ues)]
    pdp = W.exp_pdp(u0.n_taps)
    pools = torch.from_numpy(np.stack([W.rayleigh_snapshots(w.config, W.link_key(u, "dl"), per_call, 1, 1, pdp)
                                       for u in range(n_ues)])).to("cuda:0")
    per_bytes = pools[0][0].numel() * pools.element_size()
    x = torch.from_numpy(W.iq_block(w.config, 100000, 0, 1, N, "cf32")).to("cuda:0")
    y = torch.empty((n_ues, N), dtype=torch.complex64, device="cuda:0")
    ent = np.zeros(n_ues, B.TAPS_SRC_DTYPE)
    ent["ue"], ent["dir"], ent["count"] = ids, B.DIRS["dl"], per_call
    ent["src"] = pools.data_ptr() + np.arange(n_ues, dtype=np.uint64) * np.uint64(per_call * per_bytes)
    ns, xp, yp = [N] * n_ues, [x.data_ptr()] * n_ues, [y[i].data_ptr() for i in range(n_ues)]

    def call(c):
        ent["k0"] = c * per_call
        ch.set_taps_device(ent)
        ch.apply_dl(ids, ns, xp, yp)

    for c in range(warm):
        call(c)
    ch.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(calls):
        call(warm + c)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / calls
    ms, n = ch.kernel_time(1)
    ch.close()
    flop = n_ues * N * u0.n_taps * 8.0
    byts = n_ues * N * (8 + 4) + N * 8 + n_ues * per_call * u0.n_taps * 8
    return dict(dt=dt, k_us=ms * 1e3 / n if n else None, flop=flop, fir_flop=flop, bytes=byts, samples=n_ues * N,
                write_bytes=n_ues * N * 8)


def paced_run(dw, U, tune, stream, slots: int, warm: int = 20, slot_us: float = 500.0):
    """Every source resident from slot 0, slots paced at slot_us: latency
    statistics after warm untimed slots."""
    from paper_2601_08217_amd import autotune as T
    ch = dw.channel(max_ues=U, budget_bytes=4 << 30, stream=stream)
    T.apply(ch, tune)
    srv = dw.server(ch, [(0, 0)] * U, warm + slots, U, slot_us=slot_us, copy_taps=bool(tune.get("copy_taps", 0)))
    srv.run(warm)
    srv.stats(reset=True)
    srv.run(slots)
    st = srv.stats()
    srv.close()
    ch.close()
    return {k: (round(st[k], 1) if isinstance(st[k], float) else st[k])
            for k in ("lat_p50_us", "lat_p99_us", "lat_max_us", "misses", "late_starts", "start_lag_max_us",
                      "slots", "max_active")}


def c4_serving_leg(stream, slots: int, paced_slots: int):
    """C4 (64 UEs, 2x2 MIMO, 24-tap Jakes channels per antenna pair, 122.88
    Msps) served by the native slot loop: admission of every UE at slot 0
    (Jakes parameters applied at admission), back-to-back throughput with the
    convolution kernel's time, then slots paced at 0.5 ms ticks."""
    import torch
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import serving as S
    from paper_2601_08217_amd import workload as W
    w = W.workload(4)
    U = len(w.ues)
    dw = S.DeviceWorkload(w, U, x_slots=4)
    tune = T.lookup(w.name)
    ch = dw.channel(max_ues=U, budget_bytes=4 << 30, stream=stream)
    T.apply(ch, tune)
    srv = dw.server(ch, [(0, 0)] * U, 20 + slots, U)
    srv.run(20)
    ch.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.run(slots)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / slots
    ms, n = ch.kernel_time(1)
    ams, an = ch.kernel_time(2)
    srv.close()
    ch.close()
    a = dw.algorithmic()
    k_us = ms * 1e3 / n if n else None
    out = dict(workload=w.name, ues=U, value=w.link_samples_per_slot() / dt, unit="samples/s",
               us_per_slot=round(dt * 1e6, 1), k_fir_us=round(k_us, 1) if k_us else None,
               k_fir_frac_alu=round(a["fir_flop"] / (k_us * 1e-6) / PEAK_ALU, 3) if k_us else None,
               k_anchor_us=round(ams * 1e3 / an, 1) if an else None,
               flop_per_slot=a["flop"], k_fir_flop_per_slot=a["fir_flop"])
    out["paced"] = paced_run(dw, U, tune, stream, paced_slots)
    return out


def hbm_ceilings(mib: int = 1024, reps: int = 5) -> dict:
    """Bytes per second of the library's streaming probes at their best
    measured forms (one to two workgroups per CU, four 16-byte accesses in
    flight per thread): read only, write only, and copy (bytes read plus
    written).  Event-timed on the current stream."""
    import torch
    from paper_2601_08217_amd import binding as B
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.current_stream()
    out = {}
    for kind, blocks, nt in (("read", 512, False), ("write", 256, False), ("copy", 256, True)):
        d = dst.data_ptr()
        sp = 0 if kind == "write" else src.data_ptr()
        B.probe_stream(kind, d, sp, n, blocks, nt, s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            B.probe_stream(kind, d, sp, n, blocks, nt, s)
        e1.record(s)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / reps
        out[kind] = n * (2 if kind == "copy" else 1) / t
    return out


def configs_leg(stream, slots: int, only=None):
    """Every synthetic workload, back to back: UE-link samples/s and both
    roofline fractions (algorithmic FLOP against 157.3 TFLOP/s, algorithmic
    bytes against 8 TB/s), for the slot and for the convolution kernel."""
    from paper_2601_08217_amd import autotune as T
    from paper_2601_08217_amd import workload as W
    rows = []
    ceil = hbm_ceilings()
    copy_bw = ceil["copy"]
    print(f"# HBM ceilings (probes): read {ceil['read'] / 1e12:.2f}, write {ceil['write'] / 1e12:.2f}, "
          f"copy {copy_bw / 1e12:.2f} TB/s", file=sys.stderr, flush=True)
    w1 = W.workload(1)
    for name, fn in (
            ("c1_siso_dl_hold_l8", lambda: _hold_dl_direct(w1, 1, stream, 20, tune=T.lookup("c1_siso_dl_hold_l8"))),
            ("c1_dl_hold_l8_x1024ue",
             lambda: _hold_dl_direct(w1, 1024, stream, 10, tune=T.lookup("c1_dl_hold_l8_x1024ue"))),
            ("c2_4ue_dlul_linear_l16", lambda: _served(W.workload(2), stream, slots)),
            ("c3_16ue_uneven_jakes", lambda: _jakes_direct(W.workload(3), stream, slots)),
            ("c4_64ue_mimo2x2_jakes_l24", lambda: _jakes_direct(W.workload(4), stream, slots)),
            ("c5_256ue_siso_linear_l32_f16", lambda: _served(W.workload(5, tap_fmt="f16"), stream, slots))):
        if only and name not in only:
            continue
        r = fn()
        dt, k_us, flop, byts = r["dt"], r["k_us"], r["flop"], r["bytes"]
        if name.startswith("c1"):
            samples = r["samples"]
        else:
            w = W.workload(int(name[1]), tap_fmt="f16" if name.endswith("f16") else None)
            samples = w.link_samples_per_slot()
        rows.append(dict(workload=name, us_per_slot=round(dt * 1e6, 1), value=samples / dt, unit="samples/s",
                         **_roof(flop, byts, dt, k_us, r["fir_flop"]), slot_frac_copy=round(byts / dt / copy_bw, 3),
                         k_fir_frac_copy=round(byts / (k_us * 1e-6) / copy_bw, 3) if k_us else None))
        if "write_bytes" in r and k_us:
            # an output-bound launch: its writes against the write probe, and
            # its counted HBM bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE, when
            # taken on this kernel source) against 8 TB/s
            rows[-1].update(write_bytes=r["write_bytes"],
                            k_fir_frac_write_ceiling=round(r["write_bytes"] / (k_us * 1e-6) / ceil["write"], 3))
            counted = load_traffic(name, C1_TRAFFIC_FILE)
            rows[-1]["k_fir_counted_bytes"] = counted
            rows[-1]["k_fir_frac_hbm_counted"] = (round(counted / (k_us * 1e-6) / PEAK_HBM, 3)
                                                   if counted else None)
        print(f"# config {name}: {samples / dt / 1e9:.2f} G samples/s, {dt * 1e6:.1f} us per call, "
              f"bound {rows[-1]['bound']}, slot fractions ALU {rows[-1]['slot_frac_alu']} HBM "
              f"{rows[-1]['slot_frac_hbm']}", file=sys.stderr, flush=True)
    return dict(copy_probe_bytes_per_s=copy_bw, hbm_ceilings_bytes_per_s=ceil, rows=rows)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(w, n_ues: int, n_slots: int, tap_fmt: str):
    """Seeded taps and inputs of a bounded sample of the workload (cell 0, SISO)."""
    import numpy as np
    from paper_2601_08217_amd import workload as W
    u0 = w.ues[0]
    N = w.samples_per_slot(u0.sample_rate)
    K = n_slots * N // u0.period + 2
    snaps = {}
    for u in range(n_ues):
        for d in ("dl", "ul"):
            pdp = W.exp_pdp(u0.n_taps, total=1.0 if d == "dl" else 1.0 / n_ues)
            snaps[(u, d)] = W.rayleigh_snapshots(w.config, W.link_key(u, d), K, 1, 1, pdp, tap_fmt)
    pool16 = W.noise_pool(w.config, 1 << 20)
    return dict(u0=u0, N=N, n_ues=n_ues, n_slots=n_slots, tap_fmt=tap_fmt, snaps=snaps, pool16=pool16,
                dl_sigma=float(np.float32(0.1)), ul_sigma=float(np.float32(0.01)),
                xs=[[W.iq_block(w.config, u, s, 1, N, w.iq_fmt) for u in range(n_ues)] for s in range(n_slots)],
                xdl=[W.iq_block(w.config, 100000, s, 1, N, w.iq_fmt) for s in range(n_slots)])


def _oracle_on(smp, iq_fmt: str):
    """FP64 oracle over the sample: (seconds, per slot (DL outputs, UL output)), raw FP64 values."""
    import numpy as np
    from oracle import oracle as O
    from paper_2601_08217_amd import workload as W
    pool = smp["pool16"][:, 0].astype(np.float64) + 1j * smp["pool16"][:, 1].astype(np.float64)
    u0, n = smp["u0"], smp["n_ues"]
    ch = O.OracleChannel([dict(n_ant=1, ul_sigma=smp["ul_sigma"], ul_noise_off=[5])], pool, iq_fmt)
    for u in range(n):
        ch.add_ue(u, 0, u0.n_taps, 1, 1, u0.mode, period=u0.period, dl_sigma=smp["dl_sigma"],
                  dl_noise_off=[11 * u])
        for d in ("dl", "ul"):
            ch.set_taps(u, d, 0, W.taps_as_complex(smp["snaps"][(u, d)], smp["tap_fmt"]))
    ues = list(range(n))
    outs = []
    t0 = time.perf_counter()
    for s in range(smp["n_slots"]):
        y = ch.apply_dl(ues, [smp["xdl"][s]] * n, raw=True)
        z = ch.apply_ul(0, ues, smp["xs"][s], raw=True)
        outs.append((y, z))
    return time.perf_counter() - t0, outs


def _library_on(smp):
    """The library over the same sample (ci16): per slot (DL outputs, UL output) as int16 [1, N, 2]."""
    import torch
    from paper_2601_08217_amd import binding as B
    u0, n, N = smp["u0"], smp["n_ues"], smp["N"]
    ch = B.Channel([dict(sample_rate_hz=u0.sample_rate, n_ant=1, max_samples=N, ul_sigma=smp["ul_sigma"],
                         ul_noise_off=[5])], max_ues=n, hbm_budget_bytes=1 << 28, iq_fmt="ci16",
                   noise_pool=smp["pool16"])
    ids = []
    for u in range(n):
        ids.append(ch.add_ue(cell=0, n_taps=u0.n_taps, mode=u0.mode, snapshot_period=u0.period,
                             tap_fmt=smp["tap_fmt"], dl_sigma=smp["dl_sigma"], dl_noise_off=[11 * u]))
        for d in ("dl", "ul"):
            ch.set_taps(ids[-1], d, 0, smp["snaps"][(u, d)])
    outs = []
    for s in range(smp["n_slots"]):
        xdl = torch.from_numpy(smp["xdl"][s]).cuda()
        xs = [torch.from_numpy(x).cuda() for x in smp["xs"][s]]
        ys = [torch.zeros((1, N, 2), dtype=torch.int16, device="cuda") for _ in range(n)]
        z = torch.zeros((1, N, 2), dtype=torch.int16, device="cuda")
        ch.apply_dl(ids, [N] * n, [xdl.data_ptr()] * n, [y.data_ptr() for y in ys])
        ch.apply_ul(0, N, ids, [x.data_ptr() for x in xs], z.data_ptr())
        torch.cuda.synchronize()
        outs.append(([y.cpu().numpy() for y in ys], z.cpu().numpy()))
    ch.close()
    return outs


def cpu_baseline(w, n_ues: int, n_slots: int):
    """FP64 oracle on a bounded sample of the workload (n_ues UEs, n_slots
    slots, DL+UL) on every host thread, on one thread over a smaller sample,
    and the library's error against it per tap precision."""
    import numpy as np
    from oracle import oracle as O
    threads = O.num_threads()

    def timed(smp, min_s):
        # the same sample, fresh oracle state each pass, until min_s of timed work
        reps, tot = 0, 0.0
        while tot < min_s:
            dt, _ = _oracle_on(smp, w.iq_fmt)
            tot += dt
            reps += 1
        return reps, tot

    smp = _oracle_sample(w, n_ues, n_slots, w.tap_fmt)
    reps, dt = timed(smp, 10.0)
    N, L = smp["N"], smp["u0"].n_taps
    n1 = max(4, n_ues // 32)
    O.set_num_threads(1)
    try:
        reps1, dt1 = timed(_oracle_sample(w, n1, 1, w.tap_fmt), 3.0)
    finally:
        O.set_num_threads(threads)
    def versus(ref, got):
        d_max, d_cnt, n_cmp, num, den = 0, 0, 0, 0.0, 0.0
        for (ry, rz), (gy, gz) in zip(ref, got):
            for r, g in list(zip(ry, gy)) + [(rz, gz)]:
                q, _ = O.quantize_ci16(r)
                dq = np.abs(q.astype(np.int32) - g.reshape(q.shape).astype(np.int32))
                d_max, d_cnt, n_cmp = max(d_max, int(dq.max())), d_cnt + int((dq > 0).sum()), n_cmp + dq.size
                gv = O.dequantize_ci16(g.reshape(q.shape))
                num += float(np.sum(np.abs(gv - r) ** 2))
                den += float(np.sum(np.abs(r) ** 2))
        return dict(max_abs_lsb=d_max, frac_components_differing=round(d_cnt / n_cmp, 6),
                    rel_l2_vs_fp64=float(f"{(num / den) ** 0.5:.3e}"))

    # FP32 taps, and FP16 taps rounded from those same FP32 values: each
    # against the FP64 oracle fed the same stored values, and the FP16 ones
    # also against the oracle fed the FP32 values (the cost of FP16 storage)
    from paper_2601_08217_amd import workload as W
    es32 = _oracle_sample(w, 16, 2, "f32")
    es16 = dict(es32, tap_fmt="f16",
                snaps={k: W.round_taps(v.astype(np.complex128), "f16") for k, v in es32["snaps"].items()})
    _, ref32 = _oracle_on(es32, w.iq_fmt)
    _, ref16 = _oracle_on(es16, w.iq_fmt)
    got16 = _library_on(es16)
    sample = "16 UEs x 2 slots, DL+UL, ci16"
    err = {"f32": dict(versus(ref32, _library_on(es32)), sample=sample),
           "f16": dict(versus(ref16, got16), sample=sample,
                       vs_fp32_tap_oracle=versus(ref32, got16))}
    return dict(value=reps * n_slots * n_ues * N * 2 / dt, unit="samples/s", cores=threads, kind="oracle",
                sample=f"{n_ues} UEs x {n_slots} slots (DL+UL, {N} samples, L={L}) run {reps} times, {dt:.1f} s",
                single_core=dict(value=reps1 * n1 * N * 2 / dt1, unit="samples/s",
                                 sample=f"{n1} UEs x 1 slot on 1 thread, run {reps1} times, {dt1:.1f} s"),
                nproc=os.cpu_count(), cpu_model=_cpu_model(), error_vs_oracle=err)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--tap-fmt", default="f32", choices=["f32", "f16"])
    ap.add_argument("--paced-slots", type=int, default=2000)
    ap.add_argument("--plain-slots", type=int, default=8)
    ap.add_argument("--cpu-ues", type=int, default=256)
    ap.add_argument("--cpu-slots", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sparse", type=int, default=8, help="taps kept by the sparse top-n leg (0: skip)")
    ap.add_argument("--trace-period", type=int, default=30720,
                    help="snapshot period of the trace-rate leg (0: skip)")
    ap.add_argument("--mgnb-slots", type=int, default=200,
                    help="timed slots of the multi-gNB downlink leg (0: skip)")
    ap.add_argument("--trace-paths", type=int, default=24,
                    help="paths per step of the trace replay leg (0: skip)")
    ap.add_argument("--io-ues", default="64,128,192,256",
                    help="UE counts of the host IQ coupling leg ('' skips)")
    ap.add_argument("--config-slots", type=int, default=100,
                    help="slots per workload of the all-configurations leg (0: skip)")
    ap.add_argument("--configs", default="", help="workload names of the configurations leg ('': all)")
    ap.add_argument("--sweep", default="256,512,768,896,1024,1152,1280", help="UE counts of the paced sweep ('' skips)")
    ap.add_argument("--sweep-slots", type=int, default=400)
    ap.add_argument("--c4-slots", type=int, default=200,
                    help="back-to-back slots of the served C4 leg, which is then paced for --paced-slots (0: skip)")
    ap.add_argument("--pcie-slots", type=int, default=50)
    ap.add_argument("--quick", action="store_true", help="throughput only (for profiling)")
    ap.add_argument("--prime-ms", type=float, default=60.0,
                    help="untimed slots before the warm-up steps, in ms of slots (0: none)")
    ap.add_argument("--no-kernel-timing", action="store_true", help="no HIP timing events on the kernel launches (profiling)")
    ap.add_argument("--timing-every", type=int, default=4,
                    help="time the kernels of every n-th slot of the timed region (1: every slot)")
    ap.add_argument("--outputs-per-lane", type=int, default=0, choices=[0, 1, 2, 4, 8],
                    help="override the tuned outputs per lane R (0: tuned)")
    ap.add_argument("--prefetch", type=int, default=0, choices=[0, 1, 2],
                    help="override the tuned staging: 1 next item copied into LDS during the current, 2 after it "
                         "(0: tuned)")
    ap.add_argument("--dl-group", type=int, default=0, help="override the tuned DL UEs per workgroup (0: tuned)")
    ap.add_argument("--dl-subtiles", type=int, default=0, choices=[0, 1, 2, 4],
                    help="override the tuned lane tiles per DL work item (0: tuned)")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1, 2],
                    help="1: replay the slot's kernels from a captured hipGraph, 2: direct launches (0: tuned)")
    ap.add_argument("--ul-group", type=int, default=0, help="override the tuned UL UEs per workgroup (0: tuned)")
    ap.add_argument("--ul-reduce", type=int, default=0, choices=[0, 1, 2],
                    help="override the tuned UL reduction form (0: tuned, 1: fused, 2: separate pass)")
    ap.add_argument("--stream", default="own", choices=["own", "null"],
                    help="channel stream: a dedicated stream (default) or the null stream")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the channel path runs on a single MI355X here; "
              "--gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_08217_amd import serving as S
    from paper_2601_08217_amd import workload as W

    t_setup = time.perf_counter()
    w = W.workload(5, tap_fmt=args.tap_fmt)
    U = len(w.ues)
    dw = S.DeviceWorkload(w, U, x_slots=4)
    alg = dw.algorithmic()
    per_slot_samples = w.link_samples_per_slot()
    torch.cuda.synchronize()
    print(f"# setup {time.perf_counter() - t_setup:.1f} s: {w.name}, {U} UEs, {per_slot_samples} link samples/slot",
          file=sys.stderr, flush=True)

    from paper_2601_08217_amd import autotune as T
    tune = dict(T.lookup(w.name))
    if args.outputs_per_lane:
        # one R for every link, the per-class schedule set aside
        tune["outputs_per_lane"] = args.outputs_per_lane
        tune["outputs_by_class"] = {}
    if args.prefetch:
        tune["prefetch"] = args.prefetch
    if args.dl_group:
        tune["dl_group"] = args.dl_group
    if args.dl_subtiles:
        tune["dl_subtiles"] = args.dl_subtiles
    if args.graph:
        tune["graph"] = args.graph
    if args.ul_group:
        tune["ul_group"] = args.ul_group
    if args.ul_reduce:
        tune["ul_reduce"] = args.ul_reduce
    copy_taps = bool(tune.get("copy_taps", 0))
    stream = torch.cuda.Stream() if args.stream == "own" else None
    ch = dw.channel(max_ues=U, budget_bytes=1 << 30, stream=stream)
    T.apply(ch, tune)
    forever = [(0, 0)] * U
    # Setup: the GPU's clocks and the host loop reach their steady state only
    # after tens of ms of sustained slots (the first slots after an idle
    # period run the convolution 10-15% slower), so the same server first
    # runs --prime-ms of untimed slots; then come the W warm-up steps and the
    # K timed steps, back to back.
    prime = max(0, int(args.prime_ms * 1e-3 / 110e-6))
    srv = dw.server(ch, forever, prime + args.warmup + args.steps, U, copy_taps=copy_taps)
    if prime:
        srv.run(prime)
    # the warm-up slots run exactly as the timed ones do, kernel timing included
    every = 0 if args.no_kernel_timing else max(args.timing_every, 1)
    ch.enable_kernel_timing(every)
    srv.run(args.warmup)
    srv.stats(reset=True)
    ch.enable_kernel_timing(every)  # restarts the counts and the stamping period
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n = ch.kernel_time()
    kinds = {"k_fir": ch.kernel_time(1)}
    ch.enable_kernel_timing(False)
    st = srv.stats()
    srv.close()
    dt = t1 - t0
    value = args.steps * per_slot_samples / dt
    ms_per_step = 1e3 * dt / args.steps
    if k_n == 0:  # timing off: report the slot time as the launch time
        k_ms, k_n = dt * 1e3, args.steps
    fir_avg_s = (k_ms / 1e3) / max(k_n, 1)
    # the server launches one slot per step; with timing on, slots 0, every, 2*every, ... were timed
    timed_slots = -(-args.steps // every) if every else args.steps
    launches_per_step = k_n / timed_slots
    per_kind = {name: (ms * 1e3 / n if n else 0.0) for name, (ms, n) in kinds.items()}
    print(f"# batched: {value / 1e9:.1f} G samples/s, {ms_per_step * 1e3:.1f} us/slot, "
          f"{k_n} timed launches in {timed_slots} slots, kernels "
          + ", ".join(f"{k} {v:.1f} us" for k, v in per_kind.items()), file=sys.stderr, flush=True)

    flop_per_launch = alg["fir_flop"] / launches_per_step
    achieved = flop_per_launch / fir_avg_s / 1e12
    traffic = load_traffic(w.name)
    roofline = dict(bound="alu", achieved=round(achieved, 2), peak=PEAK_FP32_VECTOR_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                    traffic=traffic,
                    kernel="k_fir", flop_per_launch=flop_per_launch, launch_us=round(fir_avg_s * 1e6, 2),
                    hbm_gbs_algorithmic=round(alg["bytes"] / launches_per_step / fir_avg_s / 1e9, 1),
                    hbm_frac_algorithmic=round(alg["bytes"] / launches_per_step / fir_avg_s / 1e9 / PEAK_HBM_GBS, 4))

    out = {"metric": "emulated complex samples/sec (all UEs) + p99 slot latency vs 0.5 ms, batched vs plain",
           "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32", "data": "synthetic (seeded CN(0,1) IQ, Rayleigh exponential-PDP taps)",
           "config": {"workload": w.name, "ues": U, "taps": 32, "tap_mode": "linear P=128", "tap_fmt": args.tap_fmt,
                      "sample_rate_hz": 61.44e6, "slot_samples": 30720, "directions": "dl+ul", "iq": "ci16",
                      "link_samples_per_slot": per_slot_samples,
                      "schedule": {k: v for k, v in tune.items() if k != "us_per_slot"} or "library default",
                      "prime_slots_before_warmup": prime,
                      "host_submit_us": round(st["host_us_mean"], 1), "host_build_us": round(st["build_us_mean"], 1),
                      "host_window_wait_us": round(st["window_wait_us_mean"], 1)},
           "roofline": roofline}

    if not args.quick:
        # plain per-UE launches on the same GPU (no batching)
        srv = dw.server(ch, forever, args.plain_slots + 2, U, plain=True)
        srv.run(2)
        srv.stats(reset=True)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        srv.run(args.plain_slots)
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        pst = srv.stats()
        srv.close()
        out["plain"] = dict(value=args.plain_slots * per_slot_samples / (p1 - p0), unit="samples/s",
                            ms_per_step=1e3 * (p1 - p0) / args.plain_slots, lat_p50_us=pst["lat_p50_us"],
                            lat_p99_us=pst["lat_p99_us"])
        print(f"# plain: {out['plain']['value'] / 1e9:.2f} G samples/s", file=sys.stderr, flush=True)

        # paced serving: 0.5 ms ticks, 256 UEs resident
        lat = {}
        srv = dw.server(ch, forever, args.paced_slots, U, slot_us=500.0, copy_taps=copy_taps)
        srv.run(args.paced_slots)
        s1 = srv.stats()
        srv.close()
        lat["steady_256"] = {k: s1[k] for k in ("lat_p50_us", "lat_p99_us", "lat_max_us", "misses", "slots",
                                                "max_active")}
        # Poisson joins with 2 s mean sessions: the stated process (50/s) and
        # 128/s (mean occupancy 256), both prefilled with 256 UEs, cap 256
        for tag, rate in (("poisson_50", 50.0), ("poisson_128", 128.0)):
            ses = poisson_sessions(5, rate, 2.0, args.paced_slots, 0.5e-3, prefill=U)
            ch2 = dw.channel(max_ues=U, budget_bytes=1 << 30, stream=stream)
            T.apply(ch2, tune)
            srv = dw.server(ch2, ses, args.paced_slots, U, slot_us=500.0, copy_taps=copy_taps)
            srv.run(args.paced_slots)
            s2 = srv.stats()
            srv.close()
            ch2.close()
            lat[tag] = {k: s2[k] for k in ("lat_p50_us", "lat_p99_us", "lat_max_us", "lat_p99_full_us", "misses",
                                           "slots", "full_slots", "admitted", "left", "max_queue", "min_active",
                                           "max_active")}
        # the FP16-tap variant of the same steady load
        w16 = W.workload(5, tap_fmt="f16")
        lat["steady_256_f16"] = paced_run(S.DeviceWorkload(w16, U, x_slots=4), U, dict(T.lookup(w16.name)), stream,
                                          args.paced_slots)
        out["latency"] = dict(budget_us=500.0, **lat)
        out["lat_p50_us"] = lat["steady_256"]["lat_p50_us"]
        out["lat_p99_us"] = lat["steady_256"]["lat_p99_us"]
        print(f"# paced p50/p99 {out['lat_p50_us']:.0f}/{out['lat_p99_us']:.0f} us", file=sys.stderr, flush=True)

        if args.c4_slots > 0:
            out["c4_serving"] = c4_serving_leg(stream, args.c4_slots, args.paced_slots)
            c4 = out["c4_serving"]
            print(f"# C4 served: {c4['value'] / 1e9:.1f} G samples/s, {c4['us_per_slot']} us/slot, k_fir "
                  f"{c4['k_fir_us']} us; paced p50/p99 {c4['paced']['lat_p50_us']}/{c4['paced']['lat_p99_us']} us, "
                  f"{c4['paced']['misses']} misses", file=sys.stderr, flush=True)
        if args.sweep:
            out["ue_sweep"] = ue_sweep(dw, tune, stream, [int(v) for v in args.sweep.split(",")], args.sweep_slots)
        if args.pcie_slots > 0:
            out["pcie_inclusive"] = pcie_leg(dw, w, U, tune, stream, args.pcie_slots)
            print(f"# pcie-inclusive p50/p99 {out['pcie_inclusive']['lat_p50_us']:.0f}/"
                  f"{out['pcie_inclusive']['lat_p99_us']:.0f} us", file=sys.stderr, flush=True)
        if args.trace_period > 0:
            out["trace_rate"] = trace_rate_leg(w, U, tune, stream, min(args.steps, 200), args.trace_period)
            tr = out["trace_rate"]
            print(f"# snapshots every {args.trace_period}: {tr['value'] / 1e9:.1f} G samples/s, "
                  f"k_fir {tr['k_fir_us']} us", file=sys.stderr, flush=True)
        if args.config_slots > 0:
            out["configs"] = configs_leg(stream, args.config_slots,
                                         [v for v in args.configs.split(",") if v] or None)
        if args.io_ues:
            out["host_io"] = host_io_leg(w, U, tune, stream, min(args.steps, 200),
                                         [int(v) for v in args.io_ues.split(",")])
        if args.trace_paths > 0:
            out["trace_replay"] = trace_replay_leg(w, U, tune, stream, min(args.steps, 200), args.trace_paths)
            tr = out["trace_replay"]
            print(f"# trace replay ({args.trace_paths} paths, 1 ms steps): {tr['value'] / 1e9:.1f} G samples/s, "
                  f"{tr['us_per_slot']} us/slot, resampling {tr['resample_us_per_call']} us per call",
                  file=sys.stderr, flush=True)
        if args.mgnb_slots > 0:
            out["multi_gnb"] = multi_gnb_leg(w, U, tune, stream, dw, args.mgnb_slots)
            mg = out["multi_gnb"]
            print(f"# multi-gNB ({mg['gnbs']} gNBs, every UE hears all): {mg['value'] / 1e9:.1f} G link samples/s, "
                  f"{mg['us_per_slot']} us/slot, k_fir {mg['kernels_us']['k_fir']} us", file=sys.stderr, flush=True)
        if args.sparse > 0:
            out["sparse"] = sparse_leg(w, U, tune, stream, args.sparse, min(args.steps, 200), 20, dw)
            print(f"# sparse top-{args.sparse}: {out['sparse']['value'] / 1e9:.1f} G samples/s, rel err DL "
                  f"{out['sparse']['rel_l2_err_vs_full_dl']:.4f}", file=sys.stderr, flush=True)

    ch.close()
    if not args.no_cpu and not args.quick:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_ues, args.cpu_slots)
        cb = out["cpu_baseline"]
        print(f"# cpu oracle: {cb['value'] / 1e6:.1f} M samples/s on {cb['cores']} threads, "
              f"{cb['single_core']['value'] / 1e6:.2f} M samples/s on one ({cb['cpu_model']}); library vs "
              f"oracle: " + ", ".join(f"{k} taps max {v['max_abs_lsb']} LSB, rel L2 {v['rel_l2_vs_fp64']}"
                                      for k, v in cb["error_vs_oracle"].items())
              + f"; f16 taps vs the FP32-tap oracle: rel L2 "
                f"{cb['error_vs_oracle']['f16']['vs_fp32_tap_oracle']['rel_l2_vs_fp64']}, max "
                f"{cb['error_vs_oracle']['f16']['vs_fp32_tap_oracle']['max_abs_lsb']} LSB", file=sys.stderr,
              flush=True)
    out["paper_context"] = dict(
        note="the paper times a whole OAI stack per TTI on one CPU; no samples/s figure follows from it",
        tiny_twin_p90_tti_ms=2.0, vanilla_rfsim_multitap_p90_tti_ms=8.0, vanilla_workload="5 UEs, 10 taps",
        tiny_twin_workload="up to about 10 UEs, about 20 taps", hardware="AMD Ryzen 9 7900X desktop")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
