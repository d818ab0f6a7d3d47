"""Seeded synthetic workloads for the channel-emulation path.

This module only draws random inputs and describes workload shapes. It holds
none of the emulator's arithmetic (no convolution, no tap interpolation, no
noise addition, no quantisation of outputs); both the FP64 oracle and the HIP
library consume what it produces.

The paper measures on 3GPP TR 38.901, Sionna ray-traced and ARGOS channel
traces (Sec. IV, "Tiny-Twin compatible channel traces"), none of which is
available here.  Seeded synthetic stand-ins with the same structure replace
them: complex taps on a fixed delay grid, one snapshot per time step, with an
exponential power-delay profile (Rayleigh snapshots) or a sum-of-sinusoids
Jakes Doppler process (the paper's "Jakes-based Doppler model", Sec. IV).

Every draw comes from ``numpy.random.SeedSequence(SEED, spawn_key=key)`` with
``key = (config, purpose, ...indices)`` so that any UE, slot or snapshot can be
regenerated independently by either side of a parity test.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED = 260108217

# purposes (second element of every spawn key)
P_IQ = 1
P_TAPS = 2
P_JAKES = 3
P_NOISE = 4
P_ARRIVALS = 5
P_SHAPES = 6
P_OFFSETS = 7
P_MISC = 8
P_TRACE = 9

IQ_SCALE = 4096.0  # ci16 full scale: one LSB is 2^-12
NOISE_POOL_LEN = 1 << 23


def rng(*key: int) -> np.random.Generator:
    """Generator for one spawn key (config, purpose, indices...)."""
    return np.random.default_rng(np.random.SeedSequence(SEED, spawn_key=tuple(int(k) for k in key)))


def cn01(g: np.random.Generator, shape) -> np.ndarray:
    """CN(0,1) samples: real and imaginary parts each N(0, 1/2), float64."""
    s = np.sqrt(0.5)
    return g.normal(0.0, s, shape) + 1j * g.normal(0.0, s, shape)


# ---------------------------------------------------------------------------
# IQ streams
# ---------------------------------------------------------------------------

def to_ci16(z: np.ndarray) -> np.ndarray:
    """Complex values -> interleaved int16 [..., 2] at scale 2^12 (input encoding).

    Round half to even, clamped to the int16 range.  This encodes synthetic
    *inputs*; it is not the emulator's output quantiser.
    """
    v = np.stack([z.real, z.imag], axis=-1) * IQ_SCALE
    return np.clip(np.rint(v), -32768, 32767).astype(np.int16)


def ci16_to_complex(q: np.ndarray) -> np.ndarray:
    """Interleaved int16 [..., 2] -> complex128 (exact: I * 2^-12)."""
    q = np.asarray(q)
    return (q[..., 0].astype(np.float64) + 1j * q[..., 1].astype(np.float64)) / IQ_SCALE


def to_cf32(z: np.ndarray) -> np.ndarray:
    """Complex -> complex64 (interleaved float32 I,Q)."""
    return np.ascontiguousarray(z.astype(np.complex64))


def iq_block(config: int, stream: int, pool_index: int, n_ant: int, n: int, fmt: str) -> np.ndarray:
    """One slot-sized block of a stream's input: CN(0,1), shape [n_ant, n].

    ``fmt`` is "cf32" (complex64 [n_ant, n]) or "ci16" (int16 [n_ant, n, 2]).
    """
    z = cn01(rng(config, P_IQ, stream, pool_index), (n_ant, n))
    return to_cf32(z) if fmt == "cf32" else to_ci16(z)


# ---------------------------------------------------------------------------
# Channel taps
# ---------------------------------------------------------------------------

def exp_pdp(L: int, decay_db: float = 3.0, total: float = 1.0) -> np.ndarray:
    """Exponential power-delay profile, ``decay_db`` per tap, summing to ``total``."""
    p = 10.0 ** (-decay_db * np.arange(L) / 10.0)
    return total * p / p.sum()


def round_taps(h: np.ndarray, tap_fmt: str) -> np.ndarray:
    """Round complex taps to the storage format; returns the storage array.

    "f32" -> complex64 [..., L]; "f16" -> float16 [..., L, 2] (interleaved).
    """
    if tap_fmt == "f32":
        return np.ascontiguousarray(h.astype(np.complex64))
    if tap_fmt == "f16":
        return np.ascontiguousarray(np.stack([h.real, h.imag], axis=-1).astype(np.float16))
    raise ValueError(tap_fmt)


def taps_as_complex(stored: np.ndarray, tap_fmt: str) -> np.ndarray:
    """Stored taps (see ``round_taps``) -> complex128 with the same values."""
    if tap_fmt == "f32":
        return stored.astype(np.complex128)
    s = stored.astype(np.float64)
    return s[..., 0] + 1j * s[..., 1]


def rayleigh_snapshots(config: int, link: int, count: int, n_rx: int, n_tx: int,
                       pdp: np.ndarray, tap_fmt: str = "f32", first: int = 0) -> np.ndarray:
    """Snapshots ``first .. first+count-1`` of one link's Rayleigh tap process.

    Shape [count, n_rx, n_tx, L] (complex64) or [count, n_rx, n_tx, L, 2]
    (float16).  H_k[l] ~ CN(0, p_l), i.i.d. over k, l and antenna pairs.
    Snapshot k is drawn from its own key, so any window can be regenerated.
    """
    L = len(pdp)
    amp = np.sqrt(np.asarray(pdp, dtype=np.float64))
    out = np.empty((count, n_rx, n_tx, L), dtype=np.complex128)
    # snapshots come in chunks of 256 so large windows stay cheap to draw
    CH = 256
    k = first
    end = first + count
    while k < end:
        c0 = (k // CH) * CH
        blk = cn01(rng(config, P_TAPS, link, c0 // CH), (CH, n_rx, n_tx, L)) * amp
        lo = k - c0
        hi = min(CH, end - c0)
        out[k - first:k - first + (hi - lo)] = blk[lo:hi]
        k = c0 + hi
    return round_taps(out, tap_fmt)


@dataclasses.dataclass
class RayTrace:
    """Continuous-delay CIR trace of one link, time steps ``first ..``.

    delay [K, n_paths] seconds (FP64); gain [K, n_paths, n_rx, n_tx] complex64;
    t0 is the delay the tap grid starts at (seconds)."""
    delay: np.ndarray
    gain: np.ndarray
    t0: float


def ray_trace(config: int, link: int, count: int, n_rx: int, n_tx: int, n_paths: int, fs: float,
              first: int = 0, step_s: float = 1e-3, delay_spread_s: float = 100e-9, speed_mps: float = 8.33,
              carrier_hz: float = 3.5e9, lead_taps: int = 3, total: float = 1.0) -> RayTrace:
    """Stand-in for a ray-traced or clustered (38.901-style) CIR trace (Sec. IV).

    Fixed per link: a line-of-sight delay tau0 ~ U[0.1, 2] us; excess delays
    0 and Exp(delay_spread_s) draws, sorted; path powers exp(-excess /
    delay_spread_s) scaled to sum to ``total``; arrival cosines ~ U[-1, 1]
    giving Dopplers nu_p = speed / c * carrier * cos; per antenna pair phases
    ~ U[0, 2 pi).  At step k (time t = k step_s) path p has delay
    tau0 + excess_p - nu_p t / carrier (the path shortens as the UE moves
    toward it) and gain sqrt(power_p) exp(j (phase + 2 pi nu_p t)).  Nothing
    is drawn per step, so any window regenerates exactly.  The grid starts
    ``lead_taps`` samples before the first arrival.
    """
    g = rng(config, P_TRACE, link)
    tau0 = g.uniform(0.1e-6, 2e-6)
    excess = np.concatenate([[0.0], np.sort(g.exponential(delay_spread_s, n_paths - 1))])[:n_paths]
    power = np.exp(-excess / delay_spread_s)
    power *= total / power.sum()
    nu = speed_mps / 299792458.0 * carrier_hz * g.uniform(-1.0, 1.0, n_paths)
    phase = g.uniform(0.0, 2.0 * np.pi, (n_paths, n_rx, n_tx))
    t = (first + np.arange(count, dtype=np.float64)) * step_s
    delay = tau0 + excess[None, :] - nu[None, :] * t[:, None] / carrier_hz
    ang = phase[None] + 2.0 * np.pi * (nu[None, :] * t[:, None])[:, :, None, None]
    gain = (np.sqrt(power)[None, :, None, None] * np.exp(1j * ang)).astype(np.complex64)
    return RayTrace(np.ascontiguousarray(delay), np.ascontiguousarray(gain), float(tau0 - lead_taps / fs))


@dataclasses.dataclass
class JakesParams:
    """Per-link Jakes parameters: theta [n_rx, n_tx, L], phi [n_rx, n_tx, L, 16]."""
    doppler_hz: float
    pdp: np.ndarray
    theta: np.ndarray
    phi: np.ndarray


def jakes_params(config: int, link: int, n_rx: int, n_tx: int, pdp: np.ndarray,
                 doppler_hz: float) -> JakesParams:
    """Random angle offsets and phases, i.i.d. U[-pi, pi) per (rx, tx, tap[, sinusoid])."""
    g = rng(config, P_JAKES, link)
    L = len(pdp)
    theta = g.uniform(-math.pi, math.pi, (n_rx, n_tx, L))
    phi = g.uniform(-math.pi, math.pi, (n_rx, n_tx, L, 16))
    return JakesParams(float(doppler_hz), np.asarray(pdp, np.float64), theta, phi)


# ---------------------------------------------------------------------------
# Noise
# ---------------------------------------------------------------------------

def noise_pool(config: int = 0, n: int = NOISE_POOL_LEN) -> np.ndarray:
    """Complex FP16 CN(0,1) pool, float16 [n, 2] interleaved."""
    z = cn01(rng(config, P_NOISE, 0), n)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).astype(np.float16))


def sigma_for_snr(snr_db: float, signal_power: float = 1.0) -> np.float32:
    """Noise std (complex) for a nominal signal power; stored as float32."""
    return np.float32(math.sqrt(signal_power * 10.0 ** (-snr_db / 10.0)))


def noise_offsets(config: int, key: int, count: int, pool_len: int = NOISE_POOL_LEN) -> np.ndarray:
    return rng(config, P_OFFSETS, key).integers(0, pool_len, count).astype(np.int64)


# ---------------------------------------------------------------------------
# Arrivals (serving)
# ---------------------------------------------------------------------------

def poisson_sessions(config: int, rate_per_s: float, mean_session_s: float, horizon_s: float,
                     prefill: int = 0) -> List[Tuple[float, float]]:
    """Join times and session lengths (seconds) of a Poisson join process.

    ``prefill`` sessions start at t = 0; the rest arrive with exponential
    inter-arrival times of mean 1/rate.  Session lengths are exponential.
    """
    g = rng(config, P_ARRIVALS, 0)
    out = [(0.0, float(g.exponential(mean_session_s))) for _ in range(prefill)]
    t = 0.0
    while True:
        t += float(g.exponential(1.0 / rate_per_s))
        if t >= horizon_s:
            break
        out.append((t, float(g.exponential(mean_session_s))))
    return out


# ---------------------------------------------------------------------------
# The five synthetic workloads (shapes)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class UeShape:
    ue: int
    n_taps: int
    n_tx: int            # UE antennas
    n_rx: int            # UE antennas (DL receive)
    sample_rate: float
    mode: str            # "hold" | "linear" | "jakes"
    period: int          # snapshot period P (hold/linear)
    doppler_hz: float = 0.0


@dataclasses.dataclass
class Workload:
    name: str
    config: int
    ues: List[UeShape]
    gnb_ant: int
    slot_s: float
    n_slots: int
    iq_fmt: str          # "cf32" | "ci16"
    tap_fmt: str         # "f32" | "f16"
    directions: Tuple[str, ...]
    snr_db: float = 20.0

    def samples_per_slot(self, rate: float) -> int:
        return int(round(rate * self.slot_s))

    def cells(self) -> List[float]:
        """Distinct sample rates; each is its own cell (UL sums within a cell)."""
        return sorted({u.sample_rate for u in self.ues})

    def link_samples_per_slot(self) -> int:
        """UE-link output samples per slot over all UEs and directions."""
        tot = 0
        for u in self.ues:
            n = self.samples_per_slot(u.sample_rate)
            if "dl" in self.directions:
                tot += n * u.n_rx
            if "ul" in self.directions:
                tot += n * self.gnb_ant
        return tot


def workload(config: int, tap_fmt: Optional[str] = None, n_ues: Optional[int] = None) -> Workload:
    """The five synthetic configurations (1-based ``config``)."""
    if config == 1:
        ues = [UeShape(0, 8, 1, 1, 30.72e6, "hold", 512)]
        return Workload("c1_siso_dl_hold_l8", 1, ues, 1, 10e-3, 1, "cf32", "f32", ("dl",))
    if config == 2:
        ues = [UeShape(u, 16, 1, 1, 61.44e6, "linear", 128) for u in range(4)]
        return Workload("c2_4ue_dlul_linear_l16", 2, ues, 1, 0.5e-3, 20, "ci16", "f32", ("dl", "ul"))
    if config == 3:
        g = rng(3, P_SHAPES, 0)
        n = 16 if n_ues is None else n_ues
        Ls = g.choice([4, 8, 16, 32, 64], n)
        rates = g.choice([30.72e6, 61.44e6, 122.88e6], n)
        fds = g.uniform(5.0, 300.0, n)
        ues = [UeShape(u, int(Ls[u]), 1, 1, float(rates[u]), "jakes", 0, float(fds[u])) for u in range(n)]
        return Workload("c3_16ue_uneven_jakes", 3, ues, 1, 0.5e-3, 100, "ci16", "f32", ("dl", "ul"))
    if config == 4:
        g = rng(4, P_SHAPES, 0)
        n = 64 if n_ues is None else n_ues
        fds = g.uniform(5.0, 500.0, n)
        ues = [UeShape(u, 24, 2, 2, 122.88e6, "jakes", 0, float(fds[u])) for u in range(n)]
        return Workload("c4_64ue_mimo2x2_jakes_l24", 4, ues, 2, 0.5e-3, 200, "ci16", "f32", ("dl", "ul"))
    if config == 5:
        n = 256 if n_ues is None else n_ues
        tf = tap_fmt or "f32"
        ues = [UeShape(u, 32, 1, 1, 61.44e6, "linear", 128) for u in range(n)]
        return Workload(f"c5_256ue_siso_linear_l32_{tf}", 5, ues, 1, 0.5e-3, 1000, "ci16", tf, ("dl", "ul"))
    raise ValueError(config)


def link_key(ue: int, direction: str) -> int:
    """Stream/link index used in spawn keys: DL and UL draw independently."""
    return 2 * ue + (0 if direction == "dl" else 1)


def ul_pdp_scale(w: Workload, ue: UeShape) -> float:
    """UL tap power scale 1/(U_cell * n_tx) so the gNB sum stays near unit power."""
    n_cell = sum(1 for u in w.ues if u.sample_rate == ue.sample_rate)
    return 1.0 / (n_cell * ue.n_tx)
