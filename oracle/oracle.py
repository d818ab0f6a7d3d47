"""Python front end of the FP64 CPU oracle (tt_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the library never does.  It imports nothing from the library
package and shares no code with the HIP path.  Inputs are plain numpy arrays.

``OracleChannel`` restates the stateful semantics of a channel object in the
plainest form: per (UE, direction) a sample clock that starts at 0 when the UE
joins, the stream's previous L-1 inputs (zeros before the join), the tap
snapshots set so far keyed by snapshot index, and Jakes parameters.  Downlink
outputs are per UE (Tiny-Twin Sec. III-B: every UE convolves the gNB's raw
stream with its own channel); uplink outputs are the sum over the cell's UEs in
ascending UE id of each UE's convolved stream (same paragraph: the gNB
convolves each UE's stream independently and then aggregates), plus noise once
per gNB antenna.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tt_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "libtt_oracle.so")

HOLD, LINEAR, JAKES = 0, 1, 2
MODES = {"hold": HOLD, "linear": LINEAR, "jakes": JAKES}


class _Taps(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("L", C.c_int32), ("n_tx", C.c_int32), ("n_rx", C.c_int32),
        ("P", C.c_int64), ("kbase", C.c_int64), ("nsnap", C.c_int64),
        ("snaps", C.POINTER(C.c_double)),
        ("fd", C.c_double), ("fs", C.c_double),
        ("pdp", C.POINTER(C.c_double)), ("theta", C.POINTER(C.c_double)),
        ("phi", C.POINTER(C.c_double)),
        ("nsel", C.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (gcc -O2, no fast-math, OpenMP)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # TT_ORACLE_LIB: another build of this same source (the sanitizer test
        # loads one built with AddressSanitizer and UndefinedBehaviorSanitizer)
        path = os.environ.get("TT_ORACLE_LIB")
        if not path:
            build(force=False)
        L = C.CDLL(path or LIB)
        dp, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.tto_tap.argtypes = [C.POINTER(_Taps), C.c_int, C.c_int, C.c_int, C.c_int64, dp]
        L.tto_tap.restype = C.c_int
        L.tto_fir.argtypes = [C.POINTER(_Taps), C.c_int64, C.c_int64, dp, i64p, C.c_int64, dp]
        L.tto_fir.restype = C.c_int
        L.tto_add_noise.argtypes = [dp, C.c_int64, i64p, C.c_int64, C.c_double, dp, C.c_int64, C.c_int64]
        L.tto_add_noise.restype = None
        L.tto_quantize_ci16.argtypes = [dp, C.c_int64, C.POINTER(C.c_int16)]
        L.tto_quantize_ci16.restype = C.c_int64
        L.tto_num_threads.argtypes = []
        L.tto_num_threads.restype = C.c_int
        L.tto_set_num_threads.argtypes = [C.c_int]
        L.tto_set_num_threads.restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().tto_num_threads())


def set_num_threads(n: int):
    """OpenMP threads of the oracle's parallel loops (for timing)."""
    lib().tto_set_num_threads(int(n))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _as_pairs(z: np.ndarray) -> np.ndarray:
    """complex128 array -> contiguous float64 view [..., 2]."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    return z.view(np.float64).reshape(z.shape + (2,))


class Taps:
    """Tap description of one link (one UE and direction).

    hold/linear: ``snaps`` complex [nsnap, n_rx, n_tx, L] holding snapshots
    ``kbase .. kbase + nsnap - 1`` with period ``P``.
    jakes: ``fd``, ``fs``, ``pdp`` [L], ``theta`` [n_rx, n_tx, L], ``phi`` [..., 16].
    nsel: sparse top-n (hold/linear), 0 = every tap.
    """

    def __init__(self, mode: str, L: int, n_tx: int, n_rx: int, *, P: int = 1, kbase: int = 0,
                 snaps: Optional[np.ndarray] = None, fd: float = 0.0, fs: float = 1.0,
                 pdp=None, theta=None, phi=None, nsel: int = 0):
        self.mode, self.L, self.n_tx, self.n_rx = mode, L, n_tx, n_rx
        self.nsel = int(nsel)
        self.P, self.kbase = P, kbase
        self.snaps = None if snaps is None else _as_pairs(np.asarray(snaps).reshape(-1, n_rx, n_tx, L))
        self.fd, self.fs = float(fd), float(fs)
        self.pdp = None if pdp is None else np.ascontiguousarray(pdp, dtype=np.float64)
        self.theta = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
        self.phi = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)

    def struct(self) -> _Taps:
        s = _Taps()
        s.mode, s.L, s.n_tx, s.n_rx = MODES[self.mode], self.L, self.n_tx, self.n_rx
        s.P, s.kbase = self.P, self.kbase
        if self.snaps is not None:
            s.nsnap = self.snaps.shape[0]
            s.snaps = _dp(self.snaps)
        s.fd, s.fs = self.fd, self.fs
        s.nsel = self.nsel
        if self.pdp is not None:
            s.pdp, s.theta, s.phi = _dp(self.pdp), _dp(self.theta), _dp(self.phi)
        return s


def tap(taps: Taps, r: int, t: int, l: int, n: int) -> complex:
    out = np.zeros(2)
    st = taps.struct()
    rc = lib().tto_tap(C.byref(st), r, t, l, n, _dp(out))
    if rc != 0:
        raise ValueError("tap unavailable")
    return complex(out[0], out[1])


def fir(taps: Taps, n0: int, x_ext: np.ndarray, idx: Optional[Sequence[int]] = None) -> np.ndarray:
    """s_r[n0 + i] (complex128 [n_rx, n_out]).

    ``x_ext``: complex [n_tx, L - 1 + N]; its first L - 1 columns are the
    inputs preceding n0 (history, zeros before the join).
    """
    x = _as_pairs(np.asarray(x_ext).reshape(taps.n_tx, -1))
    N = x.shape[1] - (taps.L - 1)
    if N < 0:
        raise ValueError("x_ext shorter than L-1")
    st = taps.struct()
    if idx is None:
        n_out, ip = N, None
    else:
        idx_a = np.ascontiguousarray(idx, dtype=np.int64)
        n_out, ip = len(idx_a), idx_a.ctypes.data_as(C.POINTER(C.c_int64))
    s = np.zeros((taps.n_rx, n_out, 2))
    rc = lib().tto_fir(C.byref(st), n0, N, _dp(x), ip, n_out, _dp(s))
    if rc == -1:
        raise ValueError("missing tap snapshot")
    if rc != 0:
        raise ValueError("bad output index")
    return s[..., 0] + 1j * s[..., 1]


def add_noise(v: np.ndarray, n0: int, sigma: float, pool: np.ndarray, off: int,
              idx: Optional[Sequence[int]] = None) -> np.ndarray:
    """v + sigma * w[(off + n0 + i) mod N_pool]; ``pool`` complex128 [N_pool]."""
    a = _as_pairs(np.asarray(v).reshape(-1)).copy()
    p = _as_pairs(pool)
    if idx is None:
        ip, n_out = None, a.shape[0]
    else:
        idx_a = np.ascontiguousarray(idx, dtype=np.int64)
        ip, n_out = idx_a.ctypes.data_as(C.POINTER(C.c_int64)), len(idx_a)
    lib().tto_add_noise(_dp(a), n_out, ip, n0, float(sigma), _dp(p), p.shape[0], off)
    return (a[..., 0] + 1j * a[..., 1]).reshape(np.shape(v))


def quantize_ci16(v: np.ndarray):
    """complex -> (int16 [..., 2], saturated component count)."""
    a = _as_pairs(np.asarray(v))
    q = np.empty(a.shape, dtype=np.int16)
    nsat = lib().tto_quantize_ci16(_dp(a), a.size, q.ctypes.data_as(C.POINTER(C.c_int16)))
    return q, int(nsat)


def dequantize_ci16(q: np.ndarray) -> np.ndarray:
    """Interleaved int16 [..., 2] -> complex128, x = I * 2^-12 (exact)."""
    q = np.asarray(q)
    return (q[..., 0].astype(np.float64) + 1j * q[..., 1].astype(np.float64)) * 2.0 ** -12


def resample_cir(delay_s: np.ndarray, gain: np.ndarray, fs: float, t0_s: float, L: int) -> np.ndarray:
    """Continuous-delay CIR trace -> complex taps on a fixed delay grid (Sec. IV,
    "Tiny-Twin compatible channel traces": one snapshot per time step, taps
    uniformly spaced in delay).

    The grid holds L taps, tap l at delay t0_s + l / fs.  A path of delay tau and
    complex gain a contributes through the band-limited (ideal low-pass at fs)
    kernel: tap l receives a * sinc(fs (tau - t0_s) - l) with
    sinc(x) = sin(pi x) / (pi x).  The sinc is truncated to the grid, with no
    window.

    delay_s: [K, n_paths] seconds.  gain: [K, n_paths, n_rx, n_tx] complex.
    Returns complex128 [K, n_rx, n_tx, L]; paths are summed in index order.
    The paper states this step only in words and ships no trace, so the pins
    are the kernel's closed forms (integer and half-integer delays, energy,
    fractional-delay phase) and the linearity in paths.
    """
    delay_s = np.asarray(delay_s, dtype=np.float64)
    gain = np.asarray(gain).astype(np.complex128)
    K, n_paths = delay_s.shape
    out = np.zeros((K,) + gain.shape[2:] + (L,), dtype=np.complex128)
    l = np.arange(L, dtype=np.float64)
    for k in range(K):
        for p in range(n_paths):
            kern = np.sinc(fs * (delay_s[k, p] - t0_s) - l)
            out[k] += gain[k, p][..., None] * kern
    return out


# ---------------------------------------------------------------------------
# Stateful oracle channel
# ---------------------------------------------------------------------------

class _Link:
    def __init__(self, mode, L, n_tx, n_rx, P, nsel=0):
        self.mode, self.L, self.n_tx, self.n_rx, self.P = mode, L, n_tx, n_rx, P
        self.nsel = nsel
        self.clock = 0
        self.hist = np.zeros((n_tx, max(L - 1, 0)), dtype=np.complex128)
        self.snaps: Dict[int, np.ndarray] = {}
        self.jakes = None  # (fd, fs, pdp, theta, phi)

    def taps_for(self, n0: int, N: int) -> Taps:
        L, n_tx, n_rx = self.L, self.n_tx, self.n_rx
        if self.mode == "jakes":
            fd, fs, pdp, theta, phi = self.jakes
            return Taps("jakes", L, n_tx, n_rx, fd=fd, fs=fs, pdp=pdp, theta=theta, phi=phi)
        k_first = n0 // self.P
        k_last = (n0 + max(N, 1) - 1) // self.P + (1 if self.mode == "linear" else 0)
        arr = np.zeros((k_last - k_first + 1, n_rx, n_tx, L), dtype=np.complex128)
        for k in range(k_first, k_last + 1):
            if k not in self.snaps:
                raise ValueError(f"snapshot {k} not set")
            arr[k - k_first] = self.snaps[k]
        return Taps(self.mode, L, n_tx, n_rx, P=self.P, kbase=k_first, snaps=arr, nsel=self.nsel)

    def run(self, x: np.ndarray, idx=None) -> np.ndarray:
        """Convolve one slot of input (complex [n_tx, N]); advances the link."""
        N = x.shape[1]
        taps = self.taps_for(self.clock, N)
        x_ext = np.concatenate([self.hist, x], axis=1)
        s = fir(taps, self.clock, x_ext, idx)
        if self.L > 1:
            self.hist = x_ext[:, x_ext.shape[1] - (self.L - 1):].copy()
        self.clock += N
        return s


class OracleChannel:
    """Stateful FP64 reference of a channel object.

    cells: list of dicts {n_ant, ul_sigma, ul_noise_off: [n_ant]}.
    noise_pool: complex128 [N_pool].  iq_fmt: "cf32" | "ci16".
    """

    def __init__(self, cells: List[dict], noise_pool: np.ndarray, iq_fmt: str):
        self.cells = cells
        self.cell_clock = [0] * len(cells)
        self.pool = np.ascontiguousarray(noise_pool, dtype=np.complex128)
        self.iq_fmt = iq_fmt
        self.ues: Dict[int, dict] = {}

    def add_ue(self, ue: int, cell: int, n_taps: int, n_tx: int, n_rx: int, mode: str,
               period: int = 1, dl_sigma: float = 0.0, dl_noise_off=(0, 0, 0, 0), sparse: int = 0):
        nant = self.cells[cell]["n_ant"]
        self.ues[ue] = dict(cell=cell, dl_sigma=float(dl_sigma), dl_noise_off=list(dl_noise_off),
                            n_rx=n_rx, n_tx=n_tx,
                            dl=_Link(mode, n_taps, nant, n_rx, period, sparse),
                            ul=_Link(mode, n_taps, n_tx, nant, period, sparse))

    def remove_ue(self, ue: int):
        del self.ues[ue]

    def set_taps(self, ue: int, direction: str, k0: int, snaps_complex: np.ndarray):
        link = self.ues[ue][direction]
        for i in range(snaps_complex.shape[0]):
            link.snaps[k0 + i] = np.asarray(snaps_complex[i], dtype=np.complex128)

    def set_jakes(self, ue: int, direction: str, fd: float, fs: float, pdp, theta, phi):
        self.ues[ue][direction].jakes = (fd, fs, np.asarray(pdp, np.float64),
                                         np.asarray(theta, np.float64), np.asarray(phi, np.float64))

    def _decode(self, x) -> np.ndarray:
        return dequantize_ci16(x) if self.iq_fmt == "ci16" else np.asarray(x, dtype=np.complex128)

    def _encode(self, v):
        if self.iq_fmt == "ci16":
            return quantize_ci16(v)
        return v.astype(np.complex64), 0

    def apply_dl(self, ues: Sequence[int], xs: Sequence[np.ndarray], raw: bool = False):
        """Per UE: y_r = s_r + sigma * w[(off_r + n) mod N_pool], then encoded.

        Returns a list of outputs (encoded, or the FP64 values when ``raw``).
        """
        out = []
        for u, x in zip(ues, xs):
            st = self.ues[u]
            link = st["dl"]
            n0 = link.clock
            s = link.run(self._decode(x))
            for r in range(link.n_rx):
                s[r] = add_noise(s[r], n0, st["dl_sigma"], self.pool, st["dl_noise_off"][r])
            out.append(s if raw else self._encode(s)[0])
        return out

    def apply_ul(self, cell: int, ues: Sequence[int], xs: Sequence[np.ndarray], raw: bool = False):
        """z_r = sum over UEs (ascending id) of s_{u,r} + sigma_c * w[(off_c,r + m) mod N_pool]."""
        c = self.cells[cell]
        order = sorted(range(len(ues)), key=lambda i: ues[i])
        acc = None
        for i in order:
            s = self.ues[ues[i]]["ul"].run(self._decode(xs[i]))
            acc = s if acc is None else acc + s
        m0 = self.cell_clock[cell]
        if acc is None:
            raise ValueError("empty UL batch")
        for r in range(c["n_ant"]):
            acc[r] = add_noise(acc[r], m0, c["ul_sigma"], self.pool, c["ul_noise_off"][r])
        self.cell_clock[cell] += acc.shape[1]
        return acc if raw else self._encode(acc)[0]
