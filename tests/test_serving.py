"""GPU tests of the serving loop: queued joins, session ends, continuous
batching, and every UE's output checked alone and in the mix.

The loop serves slots of a reduced-length version of the 61.44 Msps LINEAR
workload (Sec. III-A's multi-user scalability with compute-time fidelity:
UEs join and leave while the slot keeps its schedule).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_08217_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def _workload(n_ues, L=16, slot_s=0.0625e-3, tap_fmt="f32"):
    ues = [W.UeShape(u, L, 1, 1, 61.44e6, "linear", 128) for u in range(n_ues)]
    return W.Workload("serve_test", 21, ues, 1, slot_s, 10, "ci16", tap_fmt, ("dl", "ul"))


def _oracle_link(dw, i, d, m, N):
    """UE-link output of source i, direction d, at the UE's m-th served slot."""
    u = dw.shapes[i]
    L, P = u.n_taps, u.period
    tl = dw.tap_len[i]
    pool = dw.host[("taps", i, d)]
    k0, k1 = (m * N) // P, ((m + 1) * N - 1) // P + 1
    snaps = W.taps_as_complex(np.stack([pool[k % tl] for k in range(k0, k1 + 1)]), dw.w.tap_fmt)
    taps = O.Taps("linear", L, 1, 1, P=P, kbase=k0, snaps=snaps)
    return taps


def _x_ext(blocks_at, m, L):
    x = O.dequantize_ci16(blocks_at(m))
    h = np.zeros((x.shape[0], L - 1), complex) if m == 0 else O.dequantize_ci16(blocks_at(m - 1))[:, -(L - 1):]
    return np.concatenate([h, x], axis=1)


@pytest.mark.parametrize("copy_taps", [False, True])
def test_serving_queue_sessions_and_parity(copy_taps):
    import torch
    from paper_2601_08217_amd import serving as S
    n_slots, cap = 10, 3
    w = _workload(6)
    dw = S.DeviceWorkload(w, 6, x_slots=4, y_slots=n_slots, z_slots=n_slots, keep_host=True, noise_len=1 << 18)
    sessions = [(0, 4), (0, 0), (2, 3), (3, 2), (3, 5), (5, 0)]
    ch = dw.channel(max_ues=4, budget_bytes=256 << 20)
    srv = dw.server(ch, sessions, n_slots, cap, copy_taps=copy_taps)
    srv.run(4)
    srv.run(n_slots - 4)
    st = srv.stats()
    admit, leave, active = srv.admit_slot.copy(), srv.leave_slot.copy(), srv.active.copy()
    srv.close()
    leave = np.where(leave < 0, n_slots, leave)
    # queueing behind the cap: 3 and 4 arrive at slot 3 with 3 UEs active
    assert list(admit) == [0, 0, 2, 4, 5, 6]
    assert list(leave) == [4, n_slots, 5, 6, n_slots, n_slots]
    assert active.max() == cap and st["admitted"] == 6 and st["max_queue"] >= 2
    N = dw.cell_N[0]
    pool = dw.pool16[:, 0].astype(np.float64) + 1j * dw.pool16[:, 1].astype(np.float64)
    torch.cuda.synchronize()
    ys = [t.cpu().numpy() for t in dw.dl_y[:6]]
    zs = dw.ul_z[0].cpu().numpy()
    dlx = dw.host[("dl_x", 0)]
    for j in range(6):
        cfg = dw.ue_cfg[j]
        for s in range(admit[j], leave[j]):
            m = s - admit[j]
            taps = _oracle_link(dw, j, "dl", m, N)
            x_ext = _x_ext(lambda mm: dlx[(admit[j] + mm) % dw.x_slots], m, cfg["n_taps"])
            v = O.fir(taps, m * N, x_ext)
            v[0] = O.add_noise(v[0], m * N, cfg["dl_sigma"], pool, cfg["dl_noise_off"][0])
            ref = O.quantize_ci16(v)[0]
            got = ys[j][s % dw.y_slots]
            assert np.abs(got.astype(int) - ref.astype(int)).max() <= 1, (j, s)
    cell = dw.cells[0]
    for s in range(n_slots):
        acc = np.zeros((1, N), complex)
        for j in range(6):
            if admit[j] <= s < leave[j]:
                m = s - admit[j]
                taps = _oracle_link(dw, j, "ul", m, N)
                x_ext = _x_ext(lambda mm: dw.host[("ul_x", j)][mm % dw.x_slots], m, dw.ue_cfg[j]["n_taps"])
                acc += O.fir(taps, m * N, x_ext)
        acc[0] = O.add_noise(acc[0], s * N, cell["ul_sigma"], pool, cell["ul_noise_off"][0])
        ref = O.quantize_ci16(acc)[0]
        assert np.abs(zs[s % dw.z_slots].astype(int) - ref.astype(int)).max() <= 1, s
    # alone vs in the mix: a run with stream 4 only reproduces its DL bitwise
    mix = ys[4].copy()
    ch2 = dw.channel(max_ues=4, budget_bytes=256 << 20)
    srv2 = dw.server(ch2, [(int(admit[4]), 5, 4)], n_slots, cap)
    srv2.run(n_slots)
    srv2.close()
    torch.cuda.synchronize()
    alone = dw.dl_y[0].cpu().numpy()
    for s in range(admit[4], leave[4]):
        assert np.array_equal(alone[s % dw.y_slots], mix[s % dw.y_slots]), s
    ch.close()
    ch2.close()


def test_serving_pools_shorter_than_a_slot():
    """Tap pools of 7 snapshots while a slot needs 31 (LINEAR, P = 128, 3840
    samples): the loop copies each slot's snapshots in several runs through
    the pool, and every output matches the oracle."""
    import torch
    from paper_2601_08217_amd import serving as S
    n_slots = 4
    w = _workload(2)
    dw = S.DeviceWorkload(w, 2, x_slots=2, y_slots=n_slots, z_slots=n_slots, keep_host=True, noise_len=1 << 16,
                          tap_len=7)
    ch = dw.channel(max_ues=2, budget_bytes=128 << 20)
    srv = dw.server(ch, [(0, 0), (0, 0)], n_slots, 2)
    srv.run(n_slots)
    srv.close()
    torch.cuda.synchronize()
    N = dw.cell_N[0]
    pool = dw.pool16[:, 0].astype(np.float64) + 1j * dw.pool16[:, 1].astype(np.float64)
    dlx = dw.host[("dl_x", 0)]
    cell = dw.cells[0]
    for s in range(n_slots):
        acc = np.zeros((1, N), complex)
        for j in range(2):
            cfg = dw.ue_cfg[j]
            v = O.fir(_oracle_link(dw, j, "dl", s, N), s * N, _x_ext(lambda m: dlx[m % dw.x_slots], s, cfg["n_taps"]))
            v[0] = O.add_noise(v[0], s * N, cfg["dl_sigma"], pool, cfg["dl_noise_off"][0])
            got = dw.dl_y[j][s % dw.y_slots].cpu().numpy()
            assert np.abs(got.astype(int) - O.quantize_ci16(v)[0].astype(int)).max() <= 1, (j, s)
            acc += O.fir(_oracle_link(dw, j, "ul", s, N), s * N,
                         _x_ext(lambda m: dw.host[("ul_x", j)][m % dw.x_slots], s, cfg["n_taps"]))
        acc[0] = O.add_noise(acc[0], s * N, cell["ul_sigma"], pool, cell["ul_noise_off"][0])
        z = dw.ul_z[0][s % dw.z_slots].cpu().numpy()
        assert np.abs(z.astype(int) - O.quantize_ci16(acc)[0].astype(int)).max() <= 1, s
    ch.close()


def test_serving_admission_refusal_queues_until_memory_frees():
    """An arena that holds two UEs: the third join waits until one leaves."""
    from paper_2601_08217_amd import serving as S
    w = _workload(3)
    dw = S.DeviceWorkload(w, 3, x_slots=2, y_slots=2, z_slots=2, noise_len=1 << 16)
    probe = dw.channel(max_ues=8, budget_bytes=64 << 20)
    fp = probe.footprint(**{k: v for k, v in dw.ue_cfg[0].items() if k not in ("dl_sigma", "dl_noise_off")})
    fixed = probe.stats()["arena_used"]
    probe.close()
    ch = dw.channel(max_ues=8, budget_bytes=fixed + 2 * fp + 512)
    srv = dw.server(ch, [(0, 3), (0, 0), (1, 2)], 8, 8)
    srv.run(8)
    st = srv.stats()
    admit = srv.admit_slot.copy()
    srv.close()
    ch.close()
    assert list(admit) == [0, 0, 3] and st["max_active"] == 2 and st["admitted"] == 3


def test_plain_and_batched_serving_agree():
    import torch
    from paper_2601_08217_amd import serving as S
    w = _workload(4)
    outs = []
    for plain in (False, True):
        dw = S.DeviceWorkload(w, 4, x_slots=2, y_slots=4, z_slots=4, noise_len=1 << 16)
        ch = dw.channel(max_ues=4, budget_bytes=128 << 20)
        srv = dw.server(ch, [(0, 0)] * 4, 4, 4, plain=plain)
        srv.run(4)
        srv.close()
        torch.cuda.synchronize()
        outs.append(([t.cpu().numpy() for t in dw.dl_y[:4]], dw.ul_z[0].cpu().numpy()))
        ch.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    assert np.abs(outs[0][1].astype(int) - outs[1][1].astype(int)).max() <= 1


def test_paced_loop_keeps_schedule():
    from paper_2601_08217_amd import serving as S
    w = _workload(8)
    dw = S.DeviceWorkload(w, 8, x_slots=2, noise_len=1 << 16)
    ch = dw.channel(max_ues=8, budget_bytes=128 << 20)
    srv = dw.server(ch, [(0, 0)] * 8, 200, 8, slot_us=500.0)
    srv.run(200)
    st = srv.stats()
    srv.close()
    ch.close()
    assert st["slots"] == 200 and st["lat_p99_us"] < 500.0, st
    assert 0.099 * 0.5 < st["wall_s"] < 0.2, st  # 200 ticks of 0.5 ms


def test_paced_slots_behind_their_ticks_count_as_late():
    """A 5 us slot period, far below a slot's own host and GPU time: launches
    fall further behind their ticks, and since a paced slot's latency runs
    from its tick, the lag shows as misses (budget = the period) and late
    starts."""
    from paper_2601_08217_amd import serving as S
    w = _workload(8)
    dw = S.DeviceWorkload(w, 8, x_slots=2, noise_len=1 << 16)
    ch = dw.channel(max_ues=8, budget_bytes=128 << 20)
    srv = dw.server(ch, [(0, 0)] * 8, 100, 8, slot_us=5.0)
    srv.run(100)
    st = srv.stats()
    srv.close()
    ch.close()
    assert st["slots"] == 100, st
    assert st["late_starts"] >= 50 and st["misses"] >= 50, st
    assert st["start_lag_max_us"] > 100.0 and st["lat_max_us"] >= st["start_lag_max_us"], st


def test_slot_path_allocates_no_device_memory():
    """Everything the slot path uses (descriptor buffers, the graph's
    descriptor buffer, timing events, sparse selection storage, release
    events) is allocated at create or admission: free device memory is the
    same before and after 60 served slots with kernel timing on, sparse
    top-n links, and UEs leaving and joining."""
    import torch
    from paper_2601_08217_amd import serving as S
    w = _workload(6)
    dw = S.DeviceWorkload(w, 6, x_slots=2, noise_len=1 << 16, sparse_taps=4)
    ch = dw.channel(max_ues=6, budget_bytes=128 << 20)
    ch.enable_kernel_timing(1)
    sessions = [(0, 10), (0, 0), (5, 20), (12, 0), (30, 5), (31, 0)]
    srv = dw.server(ch, sessions, 62, 4)
    srv.run(2)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    srv.run(60)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    st = srv.stats()
    srv.close()
    ms, n = ch.kernel_time(1)
    ch.close()
    assert st["admitted"] == 6 and st["left"] >= 2, st
    assert n >= 60 and ms > 0.0, (ms, n)
    assert free1 == free0, (free0, free1)
