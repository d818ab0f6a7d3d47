"""ctypes binding of libtt_channel.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/tt_channel.h
under the same name; all computation happens in the library's HIP kernels.
Device buffers are passed as integer device addresses (for example
``torch.Tensor.data_ptr()``); tap and Jakes arrays are host numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# TT_CHANNEL_LIB selects another build of the same library (same ABI), e.g.
# one compiled with different options; by default the in-tree build is used.
LIB_PATH = os.environ.get("TT_CHANNEL_LIB") or os.path.join(_PKG, "libtt_channel.so")

TT_OK, TT_E_INVALID, TT_E_NOMEM, TT_E_ADMIT, TT_E_TAPS, TT_E_DEVICE, TT_E_STATE = 0, -1, -2, -3, -4, -5, -6
TT_DL, TT_UL = 0, 1
TT_IQ_CI16, TT_IQ_CF32 = 0, 1
TT_TAP_F32, TT_TAP_F16 = 0, 1
TT_TAPS_HOLD, TT_TAPS_LINEAR, TT_TAPS_JAKES = 0, 1, 2
TT_UL_BEGIN, TT_UL_END = 1, 2
TT_MAX_ANT, TT_MAX_TAPS = 4, 64

DIRS = {"dl": TT_DL, "ul": TT_UL}
MODES = {"hold": TT_TAPS_HOLD, "linear": TT_TAPS_LINEAR, "jakes": TT_TAPS_JAKES}
IQ_FMTS = {"ci16": TT_IQ_CI16, "cf32": TT_IQ_CF32}
TAP_FMTS = {"f32": TT_TAP_F32, "f16": TT_TAP_F16}


class TTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tt error {code}: {msg}")
        self.code = code


class tt_cell_cfg(C.Structure):
    _fields_ = [("sample_rate_hz", C.c_double), ("n_ant", C.c_int32), ("max_samples", C.c_int32),
                ("ul_sigma", C.c_float), ("ul_noise_off", C.c_int64 * TT_MAX_ANT)]


class tt_channel_cfg(C.Structure):
    _fields_ = [("max_ues", C.c_int32), ("hbm_budget_bytes", C.c_int64), ("n_cells", C.c_int32),
                ("cells", C.POINTER(tt_cell_cfg)), ("iq_fmt", C.c_int32), ("noise_pool", C.c_void_p),
                ("noise_pool_len", C.c_int64), ("hip_stream", C.c_void_p), ("device", C.c_int32)]


class tt_ue_cfg(C.Structure):
    _fields_ = [("cell", C.c_int32), ("n_taps", C.c_int32), ("n_tx", C.c_int32), ("n_rx", C.c_int32),
                ("mode", C.c_int32), ("snapshot_period", C.c_int32), ("tap_fmt", C.c_int32),
                ("ring_snapshots", C.c_int32), ("dl_sigma", C.c_float),
                ("dl_noise_off", C.c_int64 * TT_MAX_ANT), ("dl_tx_streams", C.c_int32),
                ("sparse_taps", C.c_int32)]


class tt_taps_src(C.Structure):
    _fields_ = [("ue", C.c_int32), ("dir", C.c_int32), ("k0", C.c_int64), ("count", C.c_int32),
                ("src", C.c_void_p)]


# numpy view of a tt_taps_src array (the C struct pads count to 8 bytes)
TAPS_SRC_DTYPE = np.dtype({"names": ["ue", "dir", "k0", "count", "src"],
                           "formats": ["<i4", "<i4", "<i8", "<i4", "<u8"],
                           "offsets": [0, 4, 8, 16, 24], "itemsize": 32})


class tt_cir_src(C.Structure):
    _fields_ = [("ue", C.c_int32), ("dir", C.c_int32), ("k0", C.c_int64), ("count", C.c_int32),
                ("n_paths", C.c_int32), ("delay_s", C.c_void_p), ("gain", C.c_void_p), ("t0_s", C.c_double)]


# numpy view of a tt_cir_src array, for replay loops that update entries in bulk
CIR_SRC_DTYPE = np.dtype([("ue", "<i4"), ("dir", "<i4"), ("k0", "<i8"), ("count", "<i4"), ("n_paths", "<i4"),
                          ("delay_s", "<u8"), ("gain", "<u8"), ("t0_s", "<f8")])


class tt_io_cfg(C.Structure):
    _fields_ = [("cell", C.c_int32), ("n_ues", C.c_int32), ("ue", C.POINTER(C.c_int32)), ("n_samples", C.c_int32),
                ("depth", C.c_int32)]


class tt_slot(C.Structure):
    _fields_ = [("n_dl", C.c_int32), ("dl_ue", C.POINTER(C.c_int32)), ("dl_x", C.POINTER(C.c_void_p)),
                ("dl_y", C.POINTER(C.c_void_p)), ("n_ul", C.c_int32), ("ul_ue", C.POINTER(C.c_int32)),
                ("ul_x", C.POINTER(C.c_void_p)), ("ul_z", C.POINTER(C.c_void_p)),
                ("cell_samples", C.POINTER(C.c_int32)), ("dl_taps", C.POINTER(C.c_void_p)),
                ("ul_taps", C.POINTER(C.c_void_p))]


class tt_stats(C.Structure):
    _fields_ = [("saturated", C.c_int64), ("launches", C.c_int64), ("slots", C.c_int64),
                ("arena_bytes", C.c_int64), ("arena_used", C.c_int64), ("active_ues", C.c_int32),
                ("graph_captures", C.c_int64), ("graph_launches", C.c_int64)]


class tt_stream(C.Structure):
    _fields_ = [("cfg", tt_ue_cfg), ("arrive_slot", C.c_int64), ("session_slots", C.c_int64),
                ("ul_x", C.c_void_p), ("x_slots", C.c_int32), ("taps", C.c_void_p * 2), ("tap_len", C.c_int64),
                ("doppler_hz", C.c_double * 2), ("pdp", C.c_void_p * 2), ("theta", C.c_void_p * 2),
                ("phi", C.c_void_p * 2), ("dl_y", C.c_void_p), ("y_slots", C.c_int32)]


class tt_serve_cfg(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("slot_us", C.c_double), ("max_active", C.c_int32),
                ("dl_x", C.POINTER(C.c_void_p)), ("x_slots", C.c_int32), ("ul_z", C.POINTER(C.c_void_p)),
                ("z_slots", C.c_int32), ("cell_samples", C.POINTER(C.c_int32)), ("plain", C.c_int32),
                ("copy_taps", C.c_int32), ("lat_us", C.POINTER(C.c_double)), ("active", C.POINTER(C.c_int32)),
                ("admit_slot", C.POINTER(C.c_int64)), ("leave_slot", C.POINTER(C.c_int64))]


class tt_serve_stats(C.Structure):
    _fields_ = [("slots", C.c_int64), ("link_samples", C.c_int64), ("ue_slots", C.c_int64),
                ("wall_s", C.c_double), ("lat_p50_us", C.c_double), ("lat_p99_us", C.c_double),
                ("lat_max_us", C.c_double), ("lat_mean_us", C.c_double), ("lat_p99_full_us", C.c_double),
                ("full_slots", C.c_int64), ("misses", C.c_int64), ("admitted", C.c_int64), ("left", C.c_int64),
                ("queued_end", C.c_int64), ("max_queue", C.c_int64), ("max_active", C.c_int32),
                ("min_active", C.c_int32), ("host_us_mean", C.c_double), ("late_starts", C.c_int64),
                ("start_lag_max_us", C.c_double), ("build_us_mean", C.c_double),
                ("window_wait_us_mean", C.c_double)]


class tt_tuning(C.Structure):
    _fields_ = [("outputs_per_lane", C.c_int32), ("ul_group", C.c_int32), ("ul_reduce", C.c_int32),
                ("dl_group", C.c_int32), ("prefetch", C.c_int32), ("persist", C.c_int32),
                ("graph", C.c_int32), ("outputs_by_class", C.c_int32 * (3 * 4 * TT_MAX_ANT)),
                ("dl_subtiles", C.c_int32)]


# shape classes of the per-class schedule: tap mode x tap-count bucket x receive antennas
TAP_BUCKETS = (8, 16, 32, 64)


def class_key(mode: str, n_taps: int, n_rx: int) -> str:
    """Name of a link's shape class, e.g. 'linear_l32_rx1' (taps rounded up to 8, 16, 32 or 64)."""
    b = next(v for v in TAP_BUCKETS if n_taps <= v)
    return f"{mode}_l{b}_rx{n_rx}"


# name -> (argtypes)
_SIGS = {
    "tt_channel_create": [C.POINTER(tt_channel_cfg), C.POINTER(C.c_void_p)],
    "tt_channel_destroy": [C.c_void_p],
    "tt_channel_footprint": [C.c_void_p, C.POINTER(tt_ue_cfg), C.POINTER(C.c_int64)],
    "tt_channel_add_ue": [C.c_void_p, C.POINTER(tt_ue_cfg), C.POINTER(C.c_int32)],
    "tt_channel_remove_ue": [C.c_void_p, C.c_int32],
    "tt_channel_set_taps": [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_void_p],
    "tt_channel_set_taps_device": [C.c_void_p, C.c_int32, C.POINTER(tt_taps_src)],
    "tt_channel_set_taps_cir": [C.c_void_p, C.c_int32, C.c_void_p],
    "tt_channel_set_jakes": [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p],
    "tt_channel_apply_dl": [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                            C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)],
    "tt_channel_apply_ul": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                            C.POINTER(C.c_void_p), C.c_void_p, C.c_uint32],
    "tt_channel_apply_ul_noalloc": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_void_p), C.c_void_p, C.c_uint32],
    "tt_channel_apply_slot": [C.c_void_p, C.POINTER(tt_slot)],
    "tt_channel_prepare_slot": [C.c_void_p, C.POINTER(tt_slot)],
    "tt_channel_launch_prepared": [C.c_void_p],
    "tt_channel_get_stats": [C.c_void_p, C.POINTER(tt_stats)],
    "tt_channel_sync": [C.c_void_p],
    "tt_channel_enable_kernel_timing": [C.c_void_p, C.c_int32],
    "tt_channel_kernel_time": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "tt_channel_kernel_time_kind": [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "tt_channel_set_tuning": [C.c_void_p, C.c_void_p],
    "tt_server_create": [C.c_void_p, C.POINTER(tt_serve_cfg), C.c_int32, C.POINTER(tt_stream), C.POINTER(C.c_void_p)],
    "tt_server_run": [C.c_void_p, C.c_int32],
    "tt_server_stats": [C.c_void_p, C.POINTER(tt_serve_stats), C.c_int32],
    "tt_server_destroy": [C.c_void_p],
    "tt_serve": [C.c_void_p, C.POINTER(tt_serve_cfg), C.c_int32, C.POINTER(tt_stream), C.POINTER(tt_serve_stats)],
    "tt_io_create": [C.c_void_p, C.POINTER(tt_io_cfg), C.POINTER(C.c_void_p)],
    "tt_io_buffers": [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                      C.POINTER(C.c_int64)],
    "tt_io_submit": [C.c_void_p, C.c_int32],
    "tt_io_poll": [C.c_void_p, C.POINTER(C.c_int32)],
    "tt_io_wait": [C.c_void_p, C.c_int32, C.POINTER(C.c_double)],
    "tt_io_destroy": [C.c_void_p],
    "tt_probe_copy": [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p],
    "tt_probe_stream": [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p],
    "tt_probe_chunked_write": [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_void_p],
    "tt_probe_fma": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p],
}

EXPORTED = sorted(list(_SIGS) + ["tt_last_error"])

_lib = None


def load():
    """Load the in-tree library; fails loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_08217_amd.build` "
                              "(the channel path has no CPU fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = C.c_int32
        lib.tt_last_error.argtypes = []
        lib.tt_last_error.restype = C.c_char_p
        _lib = lib
    return _lib


def last_error() -> str:
    return load().tt_last_error().decode()


def _check(rc: int):
    if rc != TT_OK:
        raise TTError(rc, last_error())


def _i32(vals) -> C.Array:
    vals = list(vals)
    return (C.c_int32 * max(1, len(vals)))(*vals)


def _ptrs(vals) -> C.Array:
    vals = [int(v) if v else None for v in vals]
    return (C.c_void_p * max(1, len(vals)))(*vals)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class Channel:
    """One tt_channel: cells, UE admission, taps, and DL/UL slot calls."""

    def __init__(self, cells: Sequence[dict], max_ues: int, hbm_budget_bytes: int, iq_fmt: str,
                 noise_pool: np.ndarray, stream=None, device: int = 0):
        self.lib = load()
        self._cells = (tt_cell_cfg * len(cells))()
        for i, c in enumerate(cells):
            cc = self._cells[i]
            cc.sample_rate_hz = float(c["sample_rate_hz"])
            cc.n_ant = int(c["n_ant"])
            cc.max_samples = int(c["max_samples"])
            cc.ul_sigma = float(c.get("ul_sigma", 0.0))
            offs = list(c.get("ul_noise_off", [0] * TT_MAX_ANT)) + [0] * TT_MAX_ANT
            for r in range(TT_MAX_ANT):
                cc.ul_noise_off[r] = int(offs[r])
        pool = np.ascontiguousarray(noise_pool, dtype=np.float16).reshape(-1, 2)
        cfg = tt_channel_cfg()
        cfg.max_ues = int(max_ues)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.n_cells = len(cells)
        cfg.cells = self._cells
        cfg.iq_fmt = IQ_FMTS[iq_fmt]
        cfg.noise_pool = pool.ctypes.data
        cfg.noise_pool_len = pool.shape[0]
        cfg.hip_stream = _stream_handle(stream)
        cfg.device = int(device)
        h = C.c_void_p()
        _check(self.lib.tt_channel_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self.iq_fmt = iq_fmt

    def close(self):
        if getattr(self, "h", None):
            self.lib.tt_channel_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def ue_cfg(cell=0, n_taps=1, n_tx=1, n_rx=1, mode="hold", snapshot_period=1, tap_fmt="f32",
               ring_snapshots=0, dl_sigma=0.0, dl_noise_off=(0, 0, 0, 0), sparse_taps=0,
               dl_tx_streams=0) -> tt_ue_cfg:
        c = tt_ue_cfg()
        c.cell, c.n_taps, c.n_tx, c.n_rx = cell, n_taps, n_tx, n_rx
        c.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        c.snapshot_period = snapshot_period
        c.tap_fmt = TAP_FMTS[tap_fmt] if isinstance(tap_fmt, str) else int(tap_fmt)
        c.ring_snapshots = ring_snapshots
        c.dl_sigma = float(dl_sigma)
        offs = list(dl_noise_off) + [0] * TT_MAX_ANT
        for r in range(TT_MAX_ANT):
            c.dl_noise_off[r] = int(offs[r])
        c.sparse_taps = int(sparse_taps)
        c.dl_tx_streams = int(dl_tx_streams)
        return c

    def footprint(self, **kw) -> int:
        b = C.c_int64()
        _check(self.lib.tt_channel_footprint(self.h, C.byref(self.ue_cfg(**kw)), C.byref(b)))
        return b.value

    def add_ue(self, **kw) -> int:
        u = C.c_int32()
        _check(self.lib.tt_channel_add_ue(self.h, C.byref(self.ue_cfg(**kw)), C.byref(u)))
        return u.value

    def remove_ue(self, ue: int):
        _check(self.lib.tt_channel_remove_ue(self.h, ue))

    def set_taps(self, ue: int, direction: str, k0: int, taps: np.ndarray):
        """taps: complex64 [count, n_rx, n_tx, L] or float16 [count, n_rx, n_tx, L, 2]."""
        a = np.ascontiguousarray(taps)
        _check(self.lib.tt_channel_set_taps(self.h, ue, DIRS[direction], int(k0), int(a.shape[0]), a.ctypes.data))

    def set_taps_device(self, entries):
        """entries: (ue, direction, k0, count, device_address) tuples, or a numpy
        array of TAPS_SRC_DTYPE (dir as 0/1)."""
        if isinstance(entries, np.ndarray):
            assert entries.dtype == TAPS_SRC_DTYPE and entries.flags.c_contiguous
            _check(self.lib.tt_channel_set_taps_device(self.h, len(entries),
                                                       C.cast(entries.ctypes.data, C.POINTER(tt_taps_src))))
            return
        arr = (tt_taps_src * max(1, len(entries)))()
        for i, (ue, d, k0, count, src) in enumerate(entries):
            arr[i].ue, arr[i].dir, arr[i].k0, arr[i].count = ue, DIRS[d], int(k0), int(count)
            arr[i].src = int(src) if src else None
        _check(self.lib.tt_channel_set_taps_device(self.h, len(entries), arr))

    def set_taps_cir(self, entries):
        """Resample continuous-delay CIR steps into tap rings on the device.

        entries: a sequence of (ue, direction, k0, count, n_paths, delay_address,
        gain_address, t0_s) or a numpy array of CIR_SRC_DTYPE (dir as 0/1)."""
        if isinstance(entries, np.ndarray):
            assert entries.dtype == CIR_SRC_DTYPE and entries.flags.c_contiguous
            _check(self.lib.tt_channel_set_taps_cir(self.h, len(entries), entries.ctypes.data))
            return
        arr = (tt_cir_src * max(1, len(entries)))()
        for i, (ue, d, k0, count, n_paths, dl, g, t0) in enumerate(entries):
            arr[i].ue, arr[i].dir, arr[i].k0, arr[i].count = ue, DIRS[d], int(k0), int(count)
            arr[i].n_paths, arr[i].t0_s = int(n_paths), float(t0)
            arr[i].delay_s = int(dl) if dl else None
            arr[i].gain = int(g) if g else None
        _check(self.lib.tt_channel_set_taps_cir(self.h, len(entries), C.addressof(arr)))

    def set_jakes(self, ue: int, direction: str, doppler_hz: float, pdp, theta, phi):
        p = np.ascontiguousarray(pdp, dtype=np.float64)
        t = np.ascontiguousarray(theta, dtype=np.float64)
        f = np.ascontiguousarray(phi, dtype=np.float64)
        _check(self.lib.tt_channel_set_jakes(self.h, ue, DIRS[direction], float(doppler_hz),
                                             p.ctypes.data, t.ctypes.data, f.ctypes.data))

    def apply_dl(self, ues: Sequence[int], n_samples: Sequence[int], x: Sequence[int], y: Sequence[int]):
        _check(self.lib.tt_channel_apply_dl(self.h, len(ues), _i32(ues), _i32(n_samples), _ptrs(x), _ptrs(y)))

    def apply_ul(self, cell: int, n_samples: int, ues: Sequence[int], x: Sequence[int], z: int,
                 flags: int = TT_UL_BEGIN | TT_UL_END):
        _check(self.lib.tt_channel_apply_ul(self.h, cell, n_samples, len(ues), _i32(ues), _ptrs(x),
                                            int(z) if z else None, flags))

    def apply_ul_noalloc(self, cell: int, n_samples: int, ues: Sequence[int], x: Sequence[int], z: int,
                         flags: int = TT_UL_BEGIN | TT_UL_END):
        _check(self.lib.tt_channel_apply_ul_noalloc(self.h, cell, n_samples, len(ues), _i32(ues), _ptrs(x),
                                                    int(z) if z else None, flags))

    def apply_slot(self, dl_ues, dl_x, dl_y, ul_ues, ul_x, ul_z, cell_samples, dl_taps=None, ul_taps=None):
        self.apply_prepared(self.prepare_slot(dl_ues, dl_x, dl_y, ul_ues, ul_x, ul_z, cell_samples, dl_taps, ul_taps))

    def apply_prepared(self, prepared):
        """Submit a slot built once by ``prepare_slot`` (for loops that repeat it)."""
        _check(self.lib.tt_channel_apply_slot(self.h, C.byref(prepared[0])))

    def stage_slot(self, prepared):
        """First half of a two-step slot: validate, build the descriptors, advance the clocks."""
        _check(self.lib.tt_channel_prepare_slot(self.h, C.byref(prepared[0])))

    def launch_staged(self):
        """Second half: enqueue the staged slot."""
        _check(self.lib.tt_channel_launch_prepared(self.h))

    @staticmethod
    def prepare_slot(dl_ues, dl_x, dl_y, ul_ues, ul_x, ul_z, cell_samples, dl_taps=None, ul_taps=None):
        s = tt_slot()
        keep = [_i32(dl_ues), _ptrs(dl_x), _ptrs(dl_y), _i32(ul_ues), _ptrs(ul_x), _ptrs(ul_z), _i32(cell_samples)]
        if dl_taps is not None:
            keep.append(_ptrs(dl_taps))
            s.dl_taps = keep[-1]
        if ul_taps is not None:
            keep.append(_ptrs(ul_taps))
            s.ul_taps = keep[-1]
        s.n_dl = len(dl_ues)
        s.dl_ue, s.dl_x, s.dl_y = keep[0], keep[1], keep[2]
        s.n_ul = len(ul_ues)
        s.ul_ue, s.ul_x, s.ul_z = keep[3], keep[4], keep[5]
        s.cell_samples = keep[6]
        return s, keep

    def stats(self) -> dict:
        st = tt_stats()
        _check(self.lib.tt_channel_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in tt_stats._fields_}

    def sync(self):
        _check(self.lib.tt_channel_sync(self.h))

    def enable_kernel_timing(self, on=True):
        """False/0: off; True/1: time every slot; n > 1: every n-th slot from now on."""
        _check(self.lib.tt_channel_enable_kernel_timing(self.h, int(on)))

    def kernel_time(self, kind: int = 0):
        """(ms, launches) of timed kernels: 0 every timed span, 1 the convolution kernel,
        2 the Jakes anchor pass."""
        ms, n = C.c_double(), C.c_int64()
        _check(self.lib.tt_channel_kernel_time_kind(self.h, int(kind), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_tuning(self, outputs_per_lane: int = 0, ul_group: int = 0, ul_reduce: int = 0, dl_group: int = 0,
                   prefetch: int = 0, persist: int = 0, graph: int = 0, dl_subtiles: int = 0,
                   outputs_by_class=None):
        """outputs_by_class: {class_key(...): R} for the shape classes with their own schedule;
        dl_subtiles: lane tiles per DL work item (1, 2 or 4; 0: 1)."""
        t = tt_tuning(outputs_per_lane, ul_group, ul_reduce, dl_group, prefetch, persist, graph)
        t.dl_subtiles = int(dl_subtiles)
        for key, R in (outputs_by_class or {}).items():
            mode, lb, rx = key.split("_")
            m = MODES[mode]
            b = TAP_BUCKETS.index(int(lb[1:]))
            r = int(rx[2:]) - 1
            t.outputs_by_class[(m * 4 + b) * TT_MAX_ANT + r] = int(R)
        _check(self.lib.tt_channel_set_tuning(self.h, C.byref(t)))


class Server:
    """tt_server: the slot-paced serving loop over a Channel.

    ``streams``: list of dicts with keys cfg (kwargs of Channel.ue_cfg),
    arrive_slot, session_slots, ul_x, x_slots, taps (dl, ul device addresses),
    tap_len, jakes (per direction (doppler, pdp, theta, phi) or None), dl_y,
    y_slots.  ``dl_x``/``ul_z``: device addresses per cell.
    """

    def __init__(self, channel: Channel, streams, n_slots: int, max_active: int, dl_x, x_slots: int, ul_z,
                 z_slots: int, cell_samples, slot_us: float = 0.0, plain: bool = False, copy_taps: bool = False):
        self.lib, self.channel = channel.lib, channel
        n = len(streams)
        self._streams = (tt_stream * max(1, n))()
        self._keep = []
        for i, sd in enumerate(streams):
            st = self._streams[i]
            st.cfg = Channel.ue_cfg(**sd["cfg"])
            st.arrive_slot = int(sd.get("arrive_slot", 0))
            st.session_slots = int(sd.get("session_slots", 0))
            st.ul_x, st.x_slots = int(sd["ul_x"]), int(sd["x_slots"])
            taps = sd.get("taps") or (0, 0)
            st.taps[0], st.taps[1] = (int(taps[0]) or None), (int(taps[1]) or None)
            st.tap_len = int(sd.get("tap_len", 0))
            jk = sd.get("jakes")
            if jk:
                for d in range(2):
                    fd, pdp, theta, phi = jk[d]
                    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (pdp, theta, phi)]
                    self._keep.extend(arrs)
                    st.doppler_hz[d] = float(fd)
                    st.pdp[d], st.theta[d], st.phi[d] = (a.ctypes.data for a in arrs)
            st.dl_y, st.y_slots = int(sd["dl_y"]), int(sd["y_slots"])
        self.lat = np.full(n_slots, -1.0)
        self.active = np.zeros(n_slots, np.int32)
        self.admit_slot = np.full(max(1, n), -1, np.int64)
        self.leave_slot = np.full(max(1, n), -1, np.int64)
        self._dlx, self._ulz, self._cn = _ptrs(dl_x), _ptrs(ul_z), _i32(cell_samples)
        cfg = tt_serve_cfg()
        cfg.n_slots, cfg.slot_us, cfg.max_active = n_slots, float(slot_us), max_active
        cfg.dl_x, cfg.x_slots, cfg.ul_z, cfg.z_slots = self._dlx, x_slots, self._ulz, z_slots
        cfg.cell_samples, cfg.plain = self._cn, 1 if plain else 0
        cfg.copy_taps = 1 if copy_taps else 0
        cfg.lat_us = self.lat.ctypes.data_as(C.POINTER(C.c_double))
        cfg.active = self.active.ctypes.data_as(C.POINTER(C.c_int32))
        cfg.admit_slot = self.admit_slot.ctypes.data_as(C.POINTER(C.c_int64))
        cfg.leave_slot = self.leave_slot.ctypes.data_as(C.POINTER(C.c_int64))
        self._cfg = cfg
        h = C.c_void_p()
        _check(self.lib.tt_server_create(channel.h, C.byref(cfg), n, self._streams, C.byref(h)))
        self.h = h

    def run(self, n_slots: int):
        _check(self.lib.tt_server_run(self.h, n_slots))

    def stats(self, reset: bool = False) -> dict:
        st = tt_serve_stats()
        _check(self.lib.tt_server_stats(self.h, C.byref(st), 1 if reset else 0))
        return {k: getattr(st, k) for k, _ in tt_serve_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            rc = self.lib.tt_server_destroy(self.h)
            self.h = None
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostIO:
    """tt_io: pinned-host IQ ingress and egress around a channel's slots.

    ``inputs(b)`` / ``outputs(b)`` are numpy byte views of buffer b's pinned
    host memory (layouts in tt_channel.h)."""

    def __init__(self, channel: Channel, cell: int, ues: Sequence[int], n_samples: int, depth: int = 3):
        self.lib, self.ch = channel.lib, channel
        cfg = tt_io_cfg()
        self._ues = _i32(ues)
        cfg.cell, cfg.n_ues, cfg.ue, cfg.n_samples, cfg.depth = cell, len(ues), self._ues, n_samples, depth
        h = C.c_void_p()
        _check(self.lib.tt_io_create(channel.h, C.byref(cfg), C.byref(h)))
        self.h, self.depth = h, depth
        self._views = []
        for b in range(depth):
            pi, ni, po, no = C.c_void_p(), C.c_int64(), C.c_void_p(), C.c_int64()
            _check(self.lib.tt_io_buffers(self.h, b, C.byref(pi), C.byref(ni), C.byref(po), C.byref(no)))
            vi = np.ctypeslib.as_array((C.c_uint8 * ni.value).from_address(pi.value))
            vo = np.ctypeslib.as_array((C.c_uint8 * no.value).from_address(po.value))
            self._views.append((vi, vo))

    def inputs(self, b: int) -> np.ndarray:
        return self._views[b][0]

    def outputs(self, b: int) -> np.ndarray:
        return self._views[b][1]

    def submit(self, b: int):
        _check(self.lib.tt_io_submit(self.h, b))

    def poll(self) -> int:
        n = C.c_int32()
        _check(self.lib.tt_io_poll(self.h, C.byref(n)))
        return n.value

    def wait(self, b: int) -> float:
        lat = C.c_double()
        _check(self.lib.tt_io_wait(self.h, b, C.byref(lat)))
        return lat.value

    def close(self):
        if self.h:
            self._views = []
            _check(self.lib.tt_io_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_copy(dst: int, src: int, nbytes: int, stream=None):
    rc = load().tt_probe_copy(dst, src, nbytes, _stream_handle(stream))
    if rc != 0:
        raise TTError(TT_E_DEVICE, f"probe_copy: HIP error {rc}")


PROBE_KINDS = {"read": 0, "write": 1, "copy": 2}


def probe_stream(kind: str, dst: int, src: int, nbytes: int, blocks: int, nontemporal: bool = False, stream=None):
    rc = load().tt_probe_stream(PROBE_KINDS[kind], dst, src or None, nbytes, blocks, 1 if nontemporal else 0,
                                _stream_handle(stream))
    if rc != 0:
        raise TTError(TT_E_DEVICE if rc != 1 else TT_E_INVALID, f"probe_stream: HIP error {rc}")


def probe_chunked_write(dst: int, nbytes: int, streams: int, blocks: int, nontemporal: bool = False, stream=None):
    rc = load().tt_probe_chunked_write(dst, nbytes, streams, blocks, 1 if nontemporal else 0, _stream_handle(stream))
    if rc != 0:
        raise TTError(TT_E_DEVICE if rc != 1 else TT_E_INVALID, f"probe_chunked_write: HIP error {rc}")


def probe_fma(out: int, blocks: int, iters: int, stream=None):
    rc = load().tt_probe_fma(out, blocks, iters, _stream_handle(stream))
    if rc != 0:
        raise TTError(TT_E_DEVICE, f"probe_fma: HIP error {rc}")
