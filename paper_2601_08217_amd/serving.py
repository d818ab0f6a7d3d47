"""Device-resident sources for serving runs of the synthetic workloads.

Builds, with torch for device memory only, everything the native serving
loop (tt_server) reads: per-cell gNB input pools and UL output rings, per-UE
UL input pools, tap-snapshot pools (or Jakes parameters) and DL output rings.
All values come from the seeded generators in ``workload``.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import binding as B
from . import workload as W

DL_STREAM_BASE = 100000


class DeviceWorkload:
    """Sources for ``n_sources`` distinct UE channels of workload ``w``.

    Streams (UE sessions) map onto sources by ``stream % n_sources``; each
    stream still gets its own DL output ring.  ``sparse_taps`` > 0 runs every
    snapshot-driven UE with that many strongest taps per snapshot.
    """

    def __init__(self, w: W.Workload, n_sources: int, x_slots: int = 4, y_slots: int = 2, z_slots: int = 2,
                 device: str = "cuda:0", noise_len: int = W.NOISE_POOL_LEN, snr_db: Optional[float] = None,
                 keep_host: bool = False, sparse_taps: int = 0, tap_len: int = 0):
        import torch
        self.host = {} if keep_host else None
        self.torch, self.w, self.dev = torch, w, device
        self.x_slots, self.y_slots, self.z_slots = x_slots, y_slots, z_slots
        self.n_sources = n_sources
        self.rates = w.cells()
        self.cell_N = [w.samples_per_slot(r) for r in self.rates]
        self.n_ant = w.gnb_ant
        self.iq = w.iq_fmt
        snr = w.snr_db if snr_db is None else snr_db
        self.pool16 = W.noise_pool(w.config, noise_len)
        shapes = [w.ues[i % len(w.ues)] for i in range(n_sources)]
        self.shapes = shapes
        n_cell = [sum(1 for u in w.ues if u.sample_rate == r) for r in self.rates]
        offs = W.noise_offsets(w.config, 0, 4 * (n_sources + len(self.rates)), noise_len)
        # cells
        self.dl_x, self.ul_z, self.cells = [], [], []
        for c, r in enumerate(self.rates):
            N = self.cell_N[c]
            blocks = np.stack([W.iq_block(w.config, DL_STREAM_BASE + c, p, self.n_ant, N, self.iq)
                               for p in range(x_slots)])
            if self.host is not None:
                self.host[("dl_x", c)] = blocks
            self.dl_x.append(self._dev(blocks))
            self.ul_z.append(self._zeros((z_slots, self.n_ant, N)))
            base = 4 * (n_sources + c)
            self.cells.append(dict(sample_rate_hz=r, n_ant=self.n_ant, max_samples=N,
                                   ul_sigma=float(W.sigma_for_snr(snr, 1.0 / max(1, n_cell[c]))),
                                   ul_noise_off=[int(v) for v in offs[base:base + 4]]))
        # sources
        self.ul_x, self.taps, self.jakes, self.tap_len, self.ue_cfg = [], [], [], [], []
        for i, u in enumerate(shapes):
            c = self.rates.index(u.sample_rate)
            N = self.cell_N[c]
            blocks = np.stack([W.iq_block(w.config, i, p, u.n_tx, N, self.iq) for p in range(x_slots)])
            if self.host is not None:
                self.host[("ul_x", i)] = blocks
            self.ul_x.append(self._dev(blocks))
            pdps = {d: W.exp_pdp(u.n_taps, total=1.0 if d == "dl" else W.ul_pdp_scale(w, u)) for d in ("dl", "ul")}
            dims = {"dl": (u.n_rx, self.n_ant), "ul": (self.n_ant, u.n_tx)}
            if u.mode == "jakes":
                jk = []
                for d in ("dl", "ul"):
                    jp = W.jakes_params(w.config, W.link_key(i, d), dims[d][0], dims[d][1], pdps[d], u.doppler_hz)
                    jk.append((jp.doppler_hz, jp.pdp, jp.theta, jp.phi))
                self.jakes.append(jk)
                self.taps.append(None)
                self.tap_len.append(0)
            else:
                per_slot = N // u.period
                tl = tap_len or x_slots * per_slot  # snapshots in each pool
                tp = []
                for d in ("dl", "ul"):
                    s = W.rayleigh_snapshots(w.config, W.link_key(i, d), tl, dims[d][0], dims[d][1], pdps[d],
                                             w.tap_fmt)
                    s = np.concatenate([s, s[:1]])  # entry tap_len repeats entry 0
                    if self.host is not None:
                        self.host[("taps", i, d)] = s
                    tp.append(self._dev(s))
                self.taps.append(tp)
                self.jakes.append(None)
                self.tap_len.append(tl)
            self.ue_cfg.append(dict(cell=c, n_taps=u.n_taps, n_tx=u.n_tx, n_rx=u.n_rx, mode=u.mode,
                                    snapshot_period=max(1, u.period), tap_fmt=w.tap_fmt,
                                    dl_sigma=float(W.sigma_for_snr(snr, float(self.n_ant))),
                                    dl_noise_off=[int(v) for v in offs[4 * i:4 * i + 4]],
                                    sparse_taps=int(sparse_taps) if u.mode != "jakes" else 0))
        self.dl_y: List = []

    def _dev(self, a: np.ndarray):
        return self.torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)

    def _zeros(self, shape):
        if self.iq == "ci16":
            return self.torch.zeros(tuple(shape) + (2,), dtype=self.torch.int16, device=self.dev)
        return self.torch.zeros(tuple(shape), dtype=self.torch.complex64, device=self.dev)

    def channel(self, max_ues: int, budget_bytes: int, stream=None) -> B.Channel:
        return B.Channel(self.cells, max_ues, budget_bytes, self.iq, self.pool16, stream=stream)

    def streams(self, sessions: Sequence[Tuple[int, ...]]) -> List[dict]:
        """One stream per (arrive_slot, session_slots[, source]); by default
        stream j uses source j % n_sources."""
        out = []
        while len(self.dl_y) < len(sessions):
            j = len(self.dl_y)
            u = self.shapes[j % self.n_sources]
            N = self.cell_N[self.rates.index(u.sample_rate)]
            self.dl_y.append(self._zeros((self.y_slots, u.n_rx, N)))
        for j, ses in enumerate(sessions):
            arr, sess = ses[0], ses[1]
            i = ses[2] if len(ses) > 2 else j % self.n_sources
            sd = dict(cfg=self.ue_cfg[i], arrive_slot=int(arr), session_slots=int(sess),
                      ul_x=self.ul_x[i].data_ptr(), x_slots=self.x_slots, dl_y=self.dl_y[j].data_ptr(),
                      y_slots=self.y_slots)
            if self.taps[i] is not None:
                sd["taps"] = (self.taps[i][0].data_ptr(), self.taps[i][1].data_ptr())
                sd["tap_len"] = self.tap_len[i]
            else:
                sd["jakes"] = self.jakes[i]
            out.append(sd)
        return out

    def server(self, ch: B.Channel, sessions, n_slots: int, max_active: int, slot_us: float = 0.0,
               plain: bool = False, copy_taps: bool = False) -> B.Server:
        return B.Server(ch, self.streams(sessions), n_slots, max_active,
                        [t.data_ptr() for t in self.dl_x], self.x_slots, [t.data_ptr() for t in self.ul_z],
                        self.z_slots, self.cell_N, slot_us=slot_us, plain=plain, copy_taps=copy_taps)

    def algorithmic(self) -> Dict[str, float]:
        """Per-slot algorithmic work of all sources active: FLOP and bytes.

        FIR 8 FLOP per tap-sample; per-sample tap interpolation (LINEAR, Jakes)
        4 FLOP per tap-sample; Jakes anchors 128 FLOP per tap and anchor.
        Bytes: IQ in/out (broadcast DL input counted once per cell), noise
        4 B per output sample, taps once per snapshot (8 B fp32, 4 B fp16).
        ``fir_flop``: the convolution's share (FIR and interpolation), the
        work of the convolution kernel; ``flop`` adds the anchors.
        """
        fl, by, anc = 0.0, 0.0, 0.0
        sb = 4 if self.iq == "ci16" else 8
        tb = 4 if self.w.tap_fmt == "f16" else 8
        for N in self.cell_N:
            by += self.n_ant * N * (sb + sb + 4)  # DL broadcast in, UL sum out, UL noise
        for u in self.shapes:
            N = self.cell_N[self.rates.index(u.sample_rate)]
            by += u.n_rx * N * (sb + 4)             # DL out + DL noise
            by += u.n_tx * N * sb                   # UL in
            for d in ("dl", "ul"):
                n_rx = u.n_rx if d == "dl" else self.n_ant
                n_tx = self.n_ant if d == "dl" else u.n_tx
                ts = N * n_rx * n_tx * u.n_taps
                fl += 8 * ts
                if u.mode in ("linear", "jakes"):
                    fl += 4 * ts
                if u.mode == "jakes":
                    K = jakes_anchor_spacing(u.doppler_hz, u.sample_rate)
                    anc += 128 * n_rx * n_tx * u.n_taps * (N / K)
                else:
                    by += (N / u.period) * n_rx * n_tx * u.n_taps * tb
        return {"flop": fl + anc, "fir_flop": fl, "anchor_flop": anc, "bytes": by}


def jakes_anchor_spacing(doppler_hz: float, fs: float, bound: float = 1e-6) -> int:
    """Anchor spacing the library picks: largest power of two <= 256 with
    (w K)^2 / 8 <= bound, w = 2 pi f_D / f_s."""
    w = 2 * math.pi * doppler_hz / fs
    K = 256
    while K > 1 and (w * K) ** 2 / 8 > bound:
        K //= 2
    return K
