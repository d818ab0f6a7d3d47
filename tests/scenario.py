"""Parity harness: one seeded scenario run through the HIP library and the oracle.

Inputs come only from the seeded generators in ``paper_2601_08217_amd.workload``
(IQ blocks, Rayleigh snapshots, Jakes parameters, noise pool); the oracle side
rebuilds every slot statelessly from those inputs (explicit sample clock and
the previous slot's input tail as history), so any slot can be checked
without replaying the ones before it.  Nothing on the oracle side reads a
value produced by the HIP path.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from oracle import oracle as O
from paper_2601_08217_amd import workload as W

DL_STREAM_BASE = 100000  # IQ stream ids of the gNB broadcast streams (per cell)


@dataclasses.dataclass
class CellSpec:
    fs: float
    n_ant: int
    N: int                     # samples per slot


@dataclasses.dataclass
class UeSpec:
    cell: int
    L: int
    n_tx: int = 1
    n_rx: int = 1
    mode: str = "linear"       # hold | linear | jakes
    P: int = 128
    tap_fmt: str = "f32"
    fd: float = 0.0
    sparse: int = 0            # top-n taps per snapshot (0: every tap)
    gnbs: Tuple[int, ...] = () # other cells whose gNB streams the UE also receives (DL)
    trace: int = 0             # > 0: snapshots from a continuous-delay CIR trace with this many paths


class Scenario:
    def __init__(self, config: int, cells: Sequence[CellSpec], ues: Sequence[UeSpec], iq_fmt: str = "ci16",
                 snr_db: float = 20.0, dirs: Tuple[str, ...] = ("dl", "ul"), n_slots: int = 1,
                 pool_len: int = 1 << 20, ring: int = 0, noise: bool = True):
        self.config, self.cells, self.ues = config, list(cells), list(ues)
        self.iq_fmt, self.dirs, self.n_slots = iq_fmt, dirs, n_slots
        self.ring = ring
        self.pool16 = W.noise_pool(config, pool_len)
        self.pool = self.pool16[:, 0].astype(np.float64) + 1j * self.pool16[:, 1].astype(np.float64)
        n_cell = [sum(1 for u in self.ues if u.cell == c) for c in range(len(self.cells))]
        offs = W.noise_offsets(config, 0, 4 * (len(self.ues) + len(self.cells)), pool_len)
        self.dl_sigma, self.dl_off, self.taps, self.jakes, self.pdp = [], [], {}, {}, {}
        self.traces = {}
        for i, u in enumerate(self.ues):
            c = self.cells[u.cell]
            for d in dirs:
                scale = 1.0 if d == "dl" else 1.0 / (n_cell[u.cell] * u.n_tx)
                n_tx_l = self.dl_tx(i) if d == "dl" else u.n_tx
                n_rx_l = u.n_rx if d == "dl" else c.n_ant
                pdp = W.exp_pdp(u.L, total=scale)
                self.pdp[(i, d)] = pdp
                key = W.link_key(i, d)
                if u.mode == "jakes":
                    self.jakes[(i, d)] = W.jakes_params(config, key, n_rx_l, n_tx_l, pdp, u.fd)
                elif u.trace:
                    # one trace step per snapshot period; the oracle resamples it in FP64
                    K = n_slots * c.N // u.P + 3
                    tr = W.ray_trace(config, key, K, n_rx_l, n_tx_l, u.trace, c.fs, step_s=u.P / c.fs, total=scale)
                    self.traces[(i, d)] = tr
                    self.taps[(i, d)] = W.round_taps(O.resample_cir(tr.delay, tr.gain, c.fs, tr.t0, u.L), u.tap_fmt)
                else:
                    K = n_slots * c.N // u.P + 3
                    self.taps[(i, d)] = W.rayleigh_snapshots(config, key, K, n_rx_l, n_tx_l, pdp, u.tap_fmt)
            p_sig = c.n_ant * 1.0
            self.dl_sigma.append(float(W.sigma_for_snr(snr_db, p_sig)) if noise else 0.0)
            self.dl_off.append([int(v) for v in offs[4 * i:4 * i + 4]])
        self.ul_sigma, self.ul_off = [], []
        for ci, c in enumerate(self.cells):
            # relative to one UE's nominal received UL power (1 / U_cell)
            p1 = 1.0 / max(1, n_cell[ci])
            self.ul_sigma.append(float(W.sigma_for_snr(snr_db, p1)) if noise else 0.0)
            base = 4 * (len(self.ues) + ci)
            self.ul_off.append([int(v) for v in offs[base:base + 4]])

    # ---------------- inputs ----------------
    def dl_input(self, cell: int, slot: int) -> np.ndarray:
        c = self.cells[cell]
        return W.iq_block(self.config, DL_STREAM_BASE + cell, slot, c.n_ant, c.N, self.iq_fmt)

    def dl_tx(self, ue: int) -> int:
        """DL transmit streams: the serving cell's antennas, then every other gNB heard."""
        u = self.ues[ue]
        return self.cells[u.cell].n_ant + sum(self.cells[g].n_ant for g in u.gnbs)

    def ue_dl_input(self, ue: int, slot: int) -> np.ndarray:
        """The UE's DL input: the serving cell's stream stacked with the other gNBs' streams."""
        u = self.ues[ue]
        parts = [self.dl_input(u.cell, slot)] + [self.dl_input(g, slot) for g in u.gnbs]
        return np.concatenate(parts, axis=0) if len(parts) > 1 else parts[0]

    def ul_input(self, ue: int, slot: int) -> np.ndarray:
        u = self.ues[ue]
        return W.iq_block(self.config, ue, slot, u.n_tx, self.cells[u.cell].N, self.iq_fmt)

    def decode(self, a: np.ndarray) -> np.ndarray:
        return O.dequantize_ci16(a) if self.iq_fmt == "ci16" else np.asarray(a, np.complex128)

    def snaps_complex(self, ue: int, d: str) -> np.ndarray:
        return W.taps_as_complex(self.taps[(ue, d)], self.ues[ue].tap_fmt)

    # ---------------- oracle ----------------
    def _oracle_taps(self, ue: int, d: str, n0: int, N: int) -> O.Taps:
        u, c = self.ues[ue], self.cells[self.ues[ue].cell]
        n_tx = self.dl_tx(ue) if d == "dl" else u.n_tx
        n_rx = u.n_rx if d == "dl" else c.n_ant
        if u.mode == "jakes":
            jp = self.jakes[(ue, d)]
            return O.Taps("jakes", u.L, n_tx, n_rx, fd=jp.doppler_hz, fs=c.fs, pdp=jp.pdp, theta=jp.theta, phi=jp.phi)
        k0 = n0 // u.P
        k1 = (n0 + max(N, 1) - 1) // u.P + 1
        sn = self.snaps_complex(ue, d)[k0:k1 + 1]
        return O.Taps(u.mode, u.L, n_tx, n_rx, P=u.P, kbase=k0, snaps=sn, nsel=u.sparse)

    def _x_ext(self, ue: int, d: str, slot: int) -> np.ndarray:
        u = self.ues[ue]
        get = (lambda s: self.ue_dl_input(ue, s)) if d == "dl" else (lambda s: self.ul_input(ue, s))
        x = self.decode(get(slot))
        if u.L == 1:
            return x
        if slot == 0:
            h = np.zeros((x.shape[0], u.L - 1), complex)
        else:
            prev = self.decode(get(slot - 1))
            need = u.L - 1
            if prev.shape[1] >= need:
                h = prev[:, prev.shape[1] - need:]
            else:  # slots shorter than the history: walk further back
                parts, have, s = [prev], prev.shape[1], slot - 1
                while have < need and s > 0:
                    s -= 1
                    p = self.decode(get(s))
                    parts.insert(0, p)
                    have += p.shape[1]
                h = np.concatenate(parts, axis=1)
                if h.shape[1] < need:
                    h = np.concatenate([np.zeros((x.shape[0], need - h.shape[1]), complex), h], axis=1)
                h = h[:, h.shape[1] - need:]
        return np.concatenate([h, x], axis=1)

    def oracle_link(self, ue: int, d: str, slot: int, idx=None) -> np.ndarray:
        N = self.cells[self.ues[ue].cell].N
        n0 = slot * N
        return O.fir(self._oracle_taps(ue, d, n0, N), n0, self._x_ext(ue, d, slot), idx)

    def oracle_dl(self, ue: int, slot: int, idx=None, raw=False):
        N = self.cells[self.ues[ue].cell].N
        s = self.oracle_link(ue, "dl", slot, idx)
        for r in range(s.shape[0]):
            s[r] = O.add_noise(s[r], slot * N, self.dl_sigma[ue], self.pool, self.dl_off[ue][r], idx)
        return s if raw else self._encode(s)

    def oracle_ul(self, cell: int, slot: int, idx=None, raw=False, ues: Optional[Sequence[int]] = None):
        members = sorted(i for i, u in enumerate(self.ues) if u.cell == cell and (ues is None or i in ues))
        c = self.cells[cell]
        acc = None
        for i in members:
            s = self.oracle_link(i, "ul", slot, idx)
            acc = s if acc is None else acc + s
        if acc is None:
            n = c.N if idx is None else len(idx)
            acc = np.zeros((c.n_ant, n), complex)
        for r in range(c.n_ant):
            acc[r] = O.add_noise(acc[r], slot * c.N, self.ul_sigma[cell], self.pool, self.ul_off[cell][r], idx)
        return acc if raw else self._encode(acc)

    def _encode(self, v):
        if self.iq_fmt == "ci16":
            return O.quantize_ci16(v)[0]
        return v.astype(np.complex64)

    # ---------------- tolerance scale ----------------
    def scale_dl(self, ue: int, slot: int, idx=None) -> np.ndarray:
        """A[n] = sum |h| |x| (upper bound through |snapshots|) + |sigma w|, per rx."""
        return self._scale(ue, "dl", slot, idx, self.dl_sigma[ue], self.dl_off[ue])

    def _abs_link(self, ue, d, slot, idx):
        u, c = self.ues[ue], self.cells[self.ues[ue].cell]
        N, n0 = c.N, slot * c.N
        t = self._oracle_taps(ue, d, n0, N)
        if u.mode == "jakes":
            amp = 4.0 * np.sqrt(t.pdp)  # sum of the 16 sinusoid amplitudes
            const = np.broadcast_to(amp, (1, t.n_rx, t.n_tx, u.L)).astype(complex)
            t = O.Taps("hold", u.L, t.n_tx, t.n_rx, P=1 << 40, kbase=0, snaps=const)
        else:
            sn = np.abs(t.snaps[..., 0] + 1j * t.snaps[..., 1])
            t = O.Taps(t.mode, u.L, t.n_tx, t.n_rx, P=t.P, kbase=t.kbase, snaps=sn.astype(complex))
        return O.fir(t, n0, np.abs(self._x_ext(ue, d, slot)).astype(complex), idx).real

    def _scale(self, ue, d, slot, idx, sigma, offs):
        a = self._abs_link(ue, d, slot, idx)
        N = self.cells[self.ues[ue].cell].N
        n = np.arange(N) if idx is None else np.asarray(idx)
        for r in range(a.shape[0]):
            a[r] += sigma * np.abs(self.pool[(offs[r] + slot * N + n) % len(self.pool)])
        return a

    def scale_ul(self, cell: int, slot: int, idx=None) -> np.ndarray:
        members = [i for i, u in enumerate(self.ues) if u.cell == cell]
        c = self.cells[cell]
        n = np.arange(c.N) if idx is None else np.asarray(idx)
        a = np.zeros((c.n_ant, len(n)))
        for i in members:
            a += self._abs_link(i, "ul", slot, idx)
        for r in range(c.n_ant):
            a[r] += self.ul_sigma[cell] * np.abs(self.pool[(self.ul_off[cell][r] + slot * c.N + n) % len(self.pool)])
        return a


def check_close(got, ref, scale=None, tol=1e-5, what=""):
    """ci16: |dq| <= 1 LSB per component.  cf32: ||d|| <= tol ||ref|| and
    |d[n]| <= tol * A[n] + 1e-30 per sample (A[n] from ``scale``)."""
    got, ref = np.asarray(got), np.asarray(ref)
    if got.dtype == np.int16:
        d = np.abs(got.astype(np.int32) - ref.astype(np.int32))
        assert d.max() <= 1, f"{what}: max |dq| = {d.max()} LSB"
        return int(d.max())
    d = np.abs(got.astype(np.complex128) - ref.astype(np.complex128))
    nr = np.linalg.norm(ref.astype(np.complex128))
    assert np.linalg.norm(d) <= tol * nr + 1e-30, f"{what}: rel norm err {np.linalg.norm(d) / max(nr, 1e-300)}"
    if scale is not None:
        bad = d > tol * scale + 1e-30
        assert not bad.any(), f"{what}: {bad.sum()} samples exceed tol*A, worst ratio {(d / (scale + 1e-300)).max()}"
    return float(np.linalg.norm(d) / max(nr, 1e-300))


class GpuRun:
    """Drives a Scenario through the C ABI (device buffers from torch)."""

    def __init__(self, sc: Scenario, device: str = "cuda:0", budget: int = 1 << 30, batched: bool = True,
                 tuning: Tuple[int, ...] = (0, 0), ext_taps: bool = False, by_class=None):
        import torch
        from paper_2601_08217_amd import binding as B
        self.torch, self.B, self.sc, self.dev = torch, B, sc, device
        cells = [dict(sample_rate_hz=c.fs, n_ant=c.n_ant, max_samples=max(c.N, 1), ul_sigma=sc.ul_sigma[i],
                      ul_noise_off=sc.ul_off[i]) for i, c in enumerate(sc.cells)]
        self.ch = B.Channel(cells, max_ues=max(1, len(sc.ues)), hbm_budget_bytes=budget, iq_fmt=sc.iq_fmt,
                            noise_pool=sc.pool16)
        if any(tuning) or by_class:
            self.ch.set_tuning(*tuning, outputs_by_class=by_class)
        self.ids = []
        for i, u in enumerate(sc.ues):
            uid = self.ch.add_ue(cell=u.cell, n_taps=u.L, n_tx=u.n_tx, n_rx=u.n_rx, mode=u.mode,
                                 snapshot_period=max(u.P, 1), tap_fmt=u.tap_fmt, ring_snapshots=sc.ring,
                                 dl_sigma=sc.dl_sigma[i], dl_noise_off=sc.dl_off[i], sparse_taps=u.sparse,
                                 dl_tx_streams=sc.dl_tx(i) if u.gnbs else 0)
            self.ids.append(uid)
            for d in sc.dirs:
                if u.mode == "jakes":
                    jp = sc.jakes[(i, d)]
                    self.ch.set_jakes(uid, d, jp.doppler_hz, jp.pdp, jp.theta, jp.phi)
        self.batched = batched
        self.next_k = {}
        self.ext = None
        # continuous-delay traces resident on the device; the library resamples them
        self.trace_dev = {k: (self._to_dev(tr.delay), self._to_dev(tr.gain), tr.t0) for k, tr in sc.traces.items()}
        assert not (ext_taps and sc.traces), "caller snapshots and CIR traces are separate tests"
        if ext_taps:  # whole snapshot pools resident on the device, read in place
            self.ext = {k: self._to_dev(v) for k, v in sc.taps.items()}

    def _to_dev(self, a: np.ndarray):
        t = self.torch.from_numpy(np.ascontiguousarray(a))
        return t.to(self.dev)

    def _empty(self, n_ant: int, N: int):
        if self.sc.iq_fmt == "ci16":
            return self.torch.zeros((n_ant, N, 2), dtype=self.torch.int16, device=self.dev)
        return self.torch.zeros((n_ant, N), dtype=self.torch.complex64, device=self.dev)

    def _ext_ptr(self, i: int, d: str, slot: int) -> int:
        u = self.sc.ues[i]
        if u.mode == "jakes":
            return 0
        t = self.ext[(i, d)]
        per_bytes = t[0].numel() * t.element_size()
        k_first = (slot * self.sc.cells[u.cell].N) // u.P
        return t.data_ptr() + k_first * per_bytes

    def _feed_taps(self, slot: int):
        sc = self.sc
        if self.ext is not None:
            return
        cir = []
        for i, u in enumerate(sc.ues):
            if u.mode == "jakes":
                continue
            N = sc.cells[u.cell].N
            k_need_hi = ((slot + 1) * N - 1) // u.P + 1
            for d in sc.dirs:
                k_from = self.next_k.get((i, d), 0)
                if k_need_hi + 1 > k_from:
                    if (i, d) in self.trace_dev:
                        dl, g, t0 = self.trace_dev[(i, d)]
                        cnt, npth = k_need_hi + 1 - k_from, dl.shape[1]
                        cir.append((self.ids[i], d, k_from, cnt, npth, dl.data_ptr() + k_from * dl.stride(0) * 8,
                                    g.data_ptr() + k_from * g.stride(0) * 8, t0))
                    else:
                        arr = sc.taps[(i, d)][k_from:k_need_hi + 1]
                        self.ch.set_taps(self.ids[i], d, k_from, arr)
                    self.next_k[(i, d)] = k_need_hi + 1
        if cir:
            self.ch.set_taps_cir(cir)

    def run(self, keep_slots: Optional[Sequence[int]] = None):
        """Runs all slots; returns {("dl", ue, slot): y, ("ul", cell, slot): z} as numpy."""
        sc, torch = self.sc, self.torch
        keep = set(range(sc.n_slots) if keep_slots is None else keep_slots)
        out = {}
        for s in range(sc.n_slots):
            self._feed_taps(s)
            xdl = {c: self._to_dev(sc.dl_input(c, s)) for c in range(len(sc.cells))} if "dl" in sc.dirs else {}
            dl_ids, dl_x, dl_y, ys = [], [], [], {}
            if "dl" in sc.dirs:
                for i, u in enumerate(sc.ues):
                    y = self._empty(u.n_rx, sc.cells[u.cell].N)
                    ys[i] = y
                    dl_ids.append(self.ids[i])
                    if u.gnbs:  # this UE's own stack of gNB streams
                        xs_u = self._to_dev(sc.ue_dl_input(i, s))
                        xdl[("ue", i)] = xs_u
                        dl_x.append(xs_u.data_ptr())
                    else:
                        dl_x.append(xdl[u.cell].data_ptr())
                    dl_y.append(y.data_ptr())
            ul_ids, ul_x, zs, xul = [], [], {}, []
            if "ul" in sc.dirs:
                for i, u in enumerate(sc.ues):
                    x = self._to_dev(sc.ul_input(i, s))
                    xul.append(x)
                    ul_ids.append(self.ids[i])
                    ul_x.append(x.data_ptr())
                for c, cs in enumerate(sc.cells):
                    zs[c] = self._empty(cs.n_ant, cs.N)
            cell_n = [c.N for c in sc.cells]
            if self.batched:
                ext_dl = ext_ul = None
                if self.ext is not None:
                    ext_dl = [self._ext_ptr(i, "dl", s) for i in range(len(dl_ids))]
                    ext_ul = [self._ext_ptr(i, "ul", s) for i in range(len(ul_ids))]
                self.ch.apply_slot(dl_ids, dl_x, dl_y, ul_ids, ul_x,
                                   [zs[c].data_ptr() if c in zs else 0 for c in range(len(sc.cells))], cell_n,
                                   dl_taps=ext_dl, ul_taps=ext_ul)
            else:
                for j in range(len(dl_ids)):
                    self.ch.apply_dl([dl_ids[j]], [sc.cells[sc.ues[j].cell].N], [dl_x[j]], [dl_y[j]])
                for c, cs in enumerate(sc.cells):
                    mem = [j for j, u in enumerate(sc.ues) if u.cell == c]
                    if "ul" not in sc.dirs:
                        continue
                    for k, j in enumerate(mem):
                        fl = (self.B.TT_UL_BEGIN if k == 0 else 0) | (self.B.TT_UL_END if k == len(mem) - 1 else 0)
                        self.ch.apply_ul(c, cs.N, [ul_ids[j]], [ul_x[j]], zs[c].data_ptr(), fl)
            if s in keep:
                self.ch.sync()
                for i, y in ys.items():
                    out[("dl", i, s)] = y.cpu().numpy()
                for c, z in zs.items():
                    out[("ul", c, s)] = z.cpu().numpy()
        self.ch.sync()
        return out
