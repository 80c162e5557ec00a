"""Python binding of the rDDMC C ABI (include/rddmc.h): argument marshalling only.

Every step of the transport runs in the HIP library ``librddmc.so``; PyTorch supplies
device memory and the stream.  The library must have been built (``build()`` in
``paper_1709_10187_amd.build``); if it is missing, loading raises -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

from . import media as _media

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librddmc.so")

TIME_BINS = 128
STEP_BINS = 64
STATUS = {0: "OK", -1: "EINVAL", -2: "ESIZE", -3: "EUNSUPPORTED", -4: "ENUMERIC", -5: "EHIP"}
FLAG_DIRICHLET = 1 << 0
FLAG_KEEP_RATES = 1 << 1
FLAG_GROUPS = 1 << 2          # thin states use frequency groups (Sec. 5.3 eq. 42)
FLAG_DUST_WEIGHT = 1 << 3     # dust absorption by continuous packet weights (Sec. 2.4)
WEIGHT_FIX = float(1 << 32)   # weighted escape tallies: 2^-32 units


class RddmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Medium_t(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("n_cells", C.c_int32 * 3), ("n_bins", C.c_int32),
                ("flags", C.c_uint32), ("faces", C.c_void_p * 3), ("bin_edges", C.c_void_p),
                ("k0", C.c_void_p), ("temp", C.c_void_p), ("vel", C.c_void_p),
                ("tau_threshold", C.c_double), ("f_mu", C.c_double), ("lambda_", C.c_double),
                ("n_src", C.c_int32), ("stream", C.c_uint32), ("src_pos", C.c_void_p),
                ("src_x", C.c_void_p), ("n_packets", C.c_uint64), ("x_crit", C.c_double),
                ("dust_abs", C.c_void_p), ("dust_sca", C.c_void_p), ("src_t", C.c_void_p),
                ("n_census", C.c_int32), ("reserved1", C.c_int32), ("census", C.c_void_p)]


class Batch_t(C.Structure):
    _fields_ = [("n_clouds", C.c_int32), ("reserved0", C.c_int32), ("clouds", C.POINTER(Medium_t))]


class Run_t(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("first", C.c_uint64), ("count", C.c_uint64),
                ("max_steps", C.c_uint64), ("block", C.c_int32), ("grid", C.c_int32),
                ("chunk", C.c_int32), ("tail_lanes", C.c_int32), ("surrogate", C.c_void_p)]


class SurrogateCfg_t(C.Structure):
    _fields_ = [("tau_min", C.c_double), ("tau_max", C.c_double), ("a_min", C.c_double), ("a_max", C.c_double),
                ("dx_min", C.c_double), ("dx_max", C.c_double), ("shift_max", C.c_double),
                ("g_min", C.c_double), ("g_max", C.c_double), ("x_core", C.c_double)]


class ExitKernelCfg_t(C.Structure):
    _fields_ = [("min_steps", C.c_double), ("tail", C.c_double)]


class CloudStats_t(C.Structure):
    _fields_ = [("launched", C.c_uint64), ("escaped", C.c_uint64), ("capped", C.c_uint64),
                ("steps_total", C.c_uint64), ("steps_max", C.c_uint64), ("steps_mean", C.c_double),
                ("t_mean", C.c_double), ("t_var", C.c_double), ("n_rows", C.c_int32),
                ("n_slots", C.c_int32), ("to_mc", C.c_uint64), ("to_ddmc", C.c_uint64),
                ("reflected", C.c_uint64), ("mc_steps", C.c_uint64), ("n_pix", C.c_uint64),
                ("surrogate_calls", C.c_uint64), ("absorbed", C.c_uint64), ("escaped_w", C.c_double),
                ("t_mean_w", C.c_double), ("t_var_w", C.c_double)]


class TallyOut_t(C.Structure):
    _fields_ = [("spectrum", C.POINTER(C.c_void_p)), ("time_hist", C.POINTER(C.c_void_p)),
                ("step_hist", C.POINTER(C.c_void_p)), ("stats", C.POINTER(CloudStats_t)),
                ("pixels", C.POINTER(C.c_void_p)), ("census_bin", C.POINTER(C.c_void_p)),
                ("census_path", C.POINTER(C.c_void_p)), ("census_accel", C.POINTER(C.c_void_p)),
                ("spectrum_w", C.POINTER(C.c_void_p)), ("spectrum_w2", C.POINTER(C.c_void_p))]


ABI_VERSION = 8
CENSUS_PATH_FIX = float(1 << 24)   # residence-time units per length/c
CENSUS_ACCEL_FIX = float(1 << 24)  # eq. 18 optical-depth units


EXPORTS = ["rddmc_abi_version", "rddmc_last_error", "rddmc_table_bytes", "rddmc_tally_bytes",
           "rddmc_work_bytes", "rddmc_build_leakage", "rddmc_transport", "rddmc_transport_static", "rddmc_tally_reset",
           "rddmc_tally", "rddmc_read_tables", "rddmc_philox_fill", "rddmc_mdn_bytes", "rddmc_mdn_init",
           "rddmc_mdn_set", "rddmc_mdn_get", "rddmc_mdn_forward", "rddmc_mdn_loss_grad", "rddmc_mdn_adam",
           "rddmc_surrogate_samples", "rddmc_surrogate_bytes", "rddmc_surrogate_window", "rddmc_surrogate_attach",
           "rddmc_exitkernel_scratch_bytes", "rddmc_exitkernel_bytes", "rddmc_exitkernel_build",
           "rddmc_exitlaw_samples", "rddmc_read_redistribution"]

_lib = None


def load(path: str = LIB_PATH):
    """Load librddmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1709_10187_amd.build`")
    lib = C.CDLL(path)
    vp, sz = C.c_void_p, C.c_size_t
    lib.rddmc_abi_version.restype = C.c_int32
    if lib.rddmc_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{path} has ABI {lib.rddmc_abi_version()}, the binding expects {ABI_VERSION}: rebuild it")
    lib.rddmc_last_error.restype = C.c_char_p
    for name in ("rddmc_table_bytes", "rddmc_tally_bytes", "rddmc_work_bytes"):
        getattr(lib, name).argtypes = [C.POINTER(Batch_t), C.POINTER(sz)]
        getattr(lib, name).restype = C.c_int
    lib.rddmc_build_leakage.argtypes = [C.POINTER(Batch_t), vp, sz, vp]
    lib.rddmc_transport.argtypes = [C.POINTER(Batch_t), vp, C.POINTER(Run_t), vp, sz, vp, sz, vp]
    lib.rddmc_transport_static.argtypes = [C.POINTER(Batch_t), vp, C.POINTER(Run_t), vp, sz, vp]
    lib.rddmc_tally_reset.argtypes = [C.POINTER(Batch_t), vp, sz, vp]
    lib.rddmc_tally.argtypes = [C.POINTER(Batch_t), vp, sz, C.POINTER(TallyOut_t), vp]
    lib.rddmc_read_tables.argtypes = [C.POINTER(Batch_t), vp, C.c_int32, vp, vp, vp, vp, vp]
    lib.rddmc_read_redistribution.argtypes = [C.POINTER(Batch_t), vp, C.c_int32, vp, vp, vp]
    lib.rddmc_philox_fill.argtypes = [C.c_uint32] * 6 + [C.c_uint64, vp, vp]
    lib.rddmc_mdn_bytes.argtypes = [C.c_int64, C.POINTER(sz), C.POINTER(sz), C.POINTER(C.c_int64)]
    lib.rddmc_mdn_init.argtypes = [vp, C.c_uint64, vp]
    lib.rddmc_mdn_set.argtypes = [vp, vp, vp]
    lib.rddmc_mdn_get.argtypes = [vp, vp, vp, vp]
    lib.rddmc_mdn_forward.argtypes = [vp, vp, C.c_int64, vp, C.c_int32, vp, vp]
    lib.rddmc_mdn_loss_grad.argtypes = [vp, vp, C.c_int64, vp, vp, C.c_int32, vp, vp]
    lib.rddmc_mdn_adam.argtypes = [vp, C.c_int64, C.c_float, vp]
    cfgp = C.POINTER(SurrogateCfg_t)
    lib.rddmc_surrogate_samples.argtypes = [C.POINTER(Batch_t), vp, vp, vp, C.c_int64, C.c_uint64, C.c_uint64,
                                            vp, sz, vp, vp, vp, vp]
    lib.rddmc_surrogate_bytes.argtypes = [C.POINTER(Batch_t), cfgp, C.c_int64, C.POINTER(sz),
                                          C.POINTER(C.c_uint64)]
    lib.rddmc_surrogate_window.argtypes = [C.POINTER(Batch_t), cfgp, C.c_int32, vp]
    lib.rddmc_surrogate_attach.argtypes = [C.POINTER(Batch_t), vp, vp, vp, C.c_int64, cfgp, vp, sz, vp]
    ekp = C.POINTER(ExitKernelCfg_t)
    lib.rddmc_exitkernel_scratch_bytes.argtypes = [C.POINTER(Batch_t), C.POINTER(sz)]
    lib.rddmc_exitkernel_bytes.argtypes = [C.POINTER(Batch_t), vp, ekp, vp, sz, C.POINTER(sz), C.POINTER(C.c_uint64),
                                           vp, vp]
    lib.rddmc_exitkernel_build.argtypes = [C.POINTER(Batch_t), vp, ekp, vp, sz, vp, sz, vp]
    lib.rddmc_exitlaw_samples.argtypes = [C.POINTER(Batch_t), vp, vp, vp, vp, C.c_int64, C.c_uint64, vp, sz, vp, vp,
                                          vp]
    for name in ("rddmc_build_leakage", "rddmc_transport", "rddmc_transport_static", "rddmc_tally_reset", "rddmc_tally",
                 "rddmc_read_tables", "rddmc_philox_fill", "rddmc_mdn_bytes", "rddmc_mdn_init",
                 "rddmc_mdn_set", "rddmc_mdn_get", "rddmc_mdn_forward", "rddmc_mdn_loss_grad",
                 "rddmc_mdn_adam", "rddmc_surrogate_samples", "rddmc_surrogate_bytes",
                 "rddmc_surrogate_window", "rddmc_surrogate_attach", "rddmc_exitkernel_scratch_bytes",
                 "rddmc_exitkernel_bytes", "rddmc_exitkernel_build", "rddmc_exitlaw_samples",
                 "rddmc_read_redistribution"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise RddmcError(rc, _lib.rddmc_last_error().decode())


class Batch:
    """ctypes view of a list of ``media.Medium`` (keeps the numpy inputs alive)."""

    def __init__(self, meds: Sequence[_media.Medium], keep_rates: bool = False,
                 streams: Optional[Sequence[int]] = None):
        self.meds = list(meds)
        self.streams = list(range(len(self.meds))) if streams is None else [int(v) for v in streams]
        self._keep = []
        arr = (Medium_t * len(self.meds))()
        for i, m in enumerate(self.meds):
            s = arr[i]
            s.geometry = m.geometry
            for d in range(3):
                s.n_cells[d] = int(m.n_cells[d])
            s.n_bins = m.n_bins
            s.flags = int(m.flags) | (FLAG_KEEP_RATES if keep_rates else 0)
            for d in range(3):
                s.faces[d] = self._ptr(m.faces[d])
            s.bin_edges = self._ptr(m.bin_edges)
            s.k0 = self._ptr(m.k0)
            s.temp = self._ptr(m.temp)
            s.vel = self._ptr(m.vel) if m.vel is not None else None
            s.tau_threshold = m.tau_threshold
            s.f_mu = m.f_mu
            s.lambda_ = m.lam
            s.n_src = len(m.src_x)
            s.stream = self.streams[i]
            s.src_pos = self._ptr(np.asarray(m.src_pos, dtype=np.float64).reshape(-1, 3))
            s.src_x = self._ptr(m.src_x)
            s.n_packets = int(m.n_packets)
            s.x_crit = float(m.x_crit)
            s.dust_abs = self._ptr(m.dust_abs) if m.dust_abs is not None else None
            s.dust_sca = self._ptr(m.dust_sca) if m.dust_sca is not None else None
            s.src_t = self._ptr(np.asarray(m.src_t, dtype=np.float64).reshape(-1, 2)) if m.src_t is not None else None
            s.n_census = 0 if m.census is None else len(m.census) - 1
            s.census = self._ptr(m.census) if m.census is not None else None
        self._arr = arr
        self.c = Batch_t(len(self.meds), 0, arr)

    def _ptr(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self._keep.append(a)
        return a.ctypes.data

    def ref(self):
        return C.byref(self.c)

    def n_rows(self, i):
        return {0: 2, 1: 1, 2: 6}[self.meds[i].geometry]


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def table_bytes(b: Batch) -> int:
    lib = load()
    n = C.c_size_t()
    _check(lib.rddmc_table_bytes(b.ref(), C.byref(n)))
    return n.value


def tally_bytes(b: Batch) -> int:
    lib = load()
    n = C.c_size_t()
    _check(lib.rddmc_tally_bytes(b.ref(), C.byref(n)))
    return n.value


def work_bytes(b: Batch) -> int:
    lib = load()
    n = C.c_size_t()
    _check(lib.rddmc_work_bytes(b.ref(), C.byref(n)))
    return n.value


def build_leakage(b: Batch, d_tables, stream=None):
    lib = load()
    _check(lib.rddmc_build_leakage(b.ref(), C.c_void_p(d_tables.data_ptr()), d_tables.numel(),
                                   _stream(stream)))


def tally_reset(b: Batch, d_tally, stream=None):
    lib = load()
    _check(lib.rddmc_tally_reset(b.ref(), C.c_void_p(d_tally.data_ptr()), d_tally.numel() * d_tally.element_size(),
                                 _stream(stream)))


def transport(b: Batch, d_tables, d_tally, d_work, seed=0, first=0, count=0, max_steps=(1 << 62),
              block=0, grid=0, chunk=0, tail_lanes=0, stream=None, surrogate=None):
    lib = load()
    run = Run_t(int(seed), int(first), int(count), int(max_steps), int(block), int(grid), int(chunk),
                int(tail_lanes), C.c_void_p(surrogate.data_ptr()) if surrogate is not None else None)
    _check(lib.rddmc_transport(b.ref(), C.c_void_p(d_tables.data_ptr()), C.byref(run),
                               C.c_void_p(d_tally.data_ptr()), d_tally.numel() * d_tally.element_size(),
                               C.c_void_p(d_work.data_ptr()), d_work.numel() * d_work.element_size(),
                               _stream(stream)))


def transport_static(b: Batch, d_tables, d_tally, seed=0, first=0, count=0, max_steps=(1 << 62), block=0,
                     grid=0, chunk=0, tail_lanes=0, stream=None, surrogate=None):
    """rddmc_transport_static: the same walk with the library's own device work area (no
    caller work buffer, no allocation in the call)."""
    lib = load()
    run = Run_t(int(seed), int(first), int(count), int(max_steps), int(block), int(grid), int(chunk),
                int(tail_lanes), C.c_void_p(surrogate.data_ptr()) if surrogate is not None else None)
    _check(lib.rddmc_transport_static(b.ref(), C.c_void_p(d_tables.data_ptr()), C.byref(run),
                                      C.c_void_p(d_tally.data_ptr()), d_tally.numel() * d_tally.element_size(),
                                      _stream(stream)))


@dataclasses.dataclass
class CloudTally:
    spectrum: np.ndarray       # (n_rows, nb+2) int64
    time_hist: np.ndarray      # (TIME_BINS+2,) int64
    step_hist: np.ndarray      # (STEP_BINS,) int64
    launched: int
    escaped: int
    capped: int
    steps_total: int
    steps_max: int
    steps_mean: float
    t_mean: float
    t_var: float
    to_mc: int = 0
    to_ddmc: int = 0
    reflected: int = 0
    mc_steps: int = 0
    pixels: Optional[np.ndarray] = None   # 3D: escape counts per boundary cell (see include/rddmc.h)
    surrogate_calls: int = 0
    absorbed: int = 0
    census_bin: Optional[np.ndarray] = None    # (n_census+1, cells, bins) int64 packets per state at t_e
    census_path: Optional[np.ndarray] = None   # (n_census, cells, bins) int64 residence, 2^-24 units
    census_accel: Optional[np.ndarray] = None  # (n_census, cells) int64 eq. 18 optical-depth sums, 2^-24 units
    # continuous dust weights (FLAG_DUST_WEIGHT; census_bin then holds weights in 2^-24 units)
    spectrum_w: Optional[np.ndarray] = None    # (rows, nb+2) escaped weight
    spectrum_w2: Optional[np.ndarray] = None   # (rows, nb+2) escaped squared weight
    escaped_w: float = 0.0
    t_mean_w: float = 0.0
    t_var_w: float = 0.0


def n_pixels(m) -> int:
    if m.geometry != 2:
        return 0
    nx, ny, nz = (int(v) for v in m.n_cells)
    return 2 * (ny * nz + nx * nz + nx * ny)


def tally(b: Batch, d_tally, stream=None) -> List[CloudTally]:
    lib = load()
    n = len(b.meds)
    specs = [np.zeros((b.n_rows(i), b.meds[i].n_bins + 2), dtype=np.int64) for i in range(n)]
    th = [np.zeros(TIME_BINS + 2, dtype=np.int64) for _ in range(n)]
    sh = [np.zeros(STEP_BINS, dtype=np.int64) for _ in range(n)]
    sp_ptrs = (C.c_void_p * n)(*[a.ctypes.data for a in specs])
    th_ptrs = (C.c_void_p * n)(*[a.ctypes.data for a in th])
    sh_ptrs = (C.c_void_p * n)(*[a.ctypes.data for a in sh])
    pix = [np.zeros(n_pixels(b.meds[i]), dtype=np.int64) for i in range(n)]
    px_ptrs = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in pix])
    ncen = [0 if m.census is None else len(m.census) - 1 for m in b.meds]
    cb = [np.zeros((k + 1, m.n_cells_total, m.n_bins), dtype=np.int64) if k else np.zeros(0, dtype=np.int64)
          for k, m in zip(ncen, b.meds)]
    cp = [np.zeros((k, m.n_cells_total, m.n_bins), dtype=np.int64) if k else np.zeros(0, dtype=np.int64)
          for k, m in zip(ncen, b.meds)]
    ca = [np.zeros((k, m.n_cells_total), dtype=np.int64) if k else np.zeros(0, dtype=np.int64)
          for k, m in zip(ncen, b.meds)]
    cb_ptrs = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in cb])
    cp_ptrs = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in cp])
    ca_ptrs = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in ca])
    weighted = [bool(int(m.flags) & FLAG_DUST_WEIGHT) for m in b.meds]
    sw = [np.zeros((b.n_rows(i), b.meds[i].n_bins + 2), dtype=np.int64) if weighted[i] else np.zeros(0, np.int64)
          for i in range(n)]
    sw2 = [np.zeros_like(a) for a in sw]
    sw_ptrs = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in sw])
    sw2_ptrs = (C.c_void_p * n)(*[a.ctypes.data if a.size else None for a in sw2])
    stats = (CloudStats_t * n)()
    out = TallyOut_t(sp_ptrs, th_ptrs, sh_ptrs, stats, px_ptrs, cb_ptrs, cp_ptrs, ca_ptrs, sw_ptrs, sw2_ptrs)
    _check(lib.rddmc_tally(b.ref(), C.c_void_p(d_tally.data_ptr()), d_tally.numel() * d_tally.element_size(),
                           C.byref(out), _stream(stream)))
    res = []
    for i in range(n):
        z = stats[i]
        res.append(CloudTally(specs[i], th[i], sh[i], z.launched, z.escaped, z.capped, z.steps_total,
                              z.steps_max, z.steps_mean, z.t_mean, z.t_var, z.to_mc, z.to_ddmc, z.reflected,
                              z.mc_steps, pix[i] if pix[i].size else None, z.surrogate_calls, z.absorbed,
                              cb[i] if cb[i].size else None, cp[i] if cp[i].size else None,
                              ca[i] if ca[i].size else None,
                              sw[i].astype(np.float64) / WEIGHT_FIX if weighted[i] else None,
                              sw2[i].astype(np.float64) / WEIGHT_FIX if weighted[i] else None,
                              z.escaped_w, z.t_mean_w, z.t_var_w))
    return res


HOT_DTYPE = np.dtype([("ln2_over_K", "<f4"), ("d_hi", "<u4"), ("s_hi", "<u4"), ("f_hi", "<u4")])


def read_tables(b: Batch, d_tables, cloud=0, want_rates=True, stream=None):
    """FP64 k_ij, FP64 rates (if kept), hot records and the u64 thresholds D, S, F per state."""
    lib = load()
    m = b.meds[cloud]
    ns = m.n_cells_total * m.n_bins
    nf = 6 if m.geometry == 2 else 2
    k = np.zeros(ns)
    rates = np.zeros((ns, nf + 2)) if want_rates else None
    hot = np.zeros(ns, dtype=HOT_DTYPE)
    lo = np.zeros((ns, 4), dtype=np.uint32)
    _check(lib.rddmc_read_tables(b.ref(), C.c_void_p(d_tables.data_ptr()), cloud, k.ctypes.data,
                                 rates.ctypes.data if want_rates else None, hot.ctypes.data,
                                 lo.ctypes.data, _stream(stream)))
    D = (hot["d_hi"].astype(np.uint64) << np.uint64(32)) | lo[:, 0].astype(np.uint64)
    S = (hot["s_hi"].astype(np.uint64) << np.uint64(32)) | lo[:, 1].astype(np.uint64)
    F = (hot["f_hi"].astype(np.uint64) << np.uint64(32)) | lo[:, 2].astype(np.uint64)
    return k, rates, hot, D, S, F


def read_redistribution(b: Batch, d_tables, cloud=0, stream=None):
    """Frequency-group tables of a cloud: P(j | j') [nb, nb] (row j') and the alias tables
    [nb, nb] of (threshold, alias bin)."""
    lib = load()
    nb = b.meds[cloud].n_bins
    prob = np.zeros((nb, nb))
    alias = np.zeros((nb, nb, 2), dtype=np.uint32)
    _check(lib.rddmc_read_redistribution(b.ref(), C.c_void_p(d_tables.data_ptr()), cloud, prob.ctypes.data,
                                         alias.ctypes.data, _stream(stream)))
    return prob, alias


def philox_fill(k0, k1, c0, c1, c2, c3, n, d_out, stream=None):
    lib = load()
    _check(lib.rddmc_philox_fill(k0, k1, c0, c1, c2, c3, n, C.c_void_p(d_out.data_ptr()), _stream(stream)))


class ExitKernel:
    """The exact per-cell exit kernel of a Problem's batch (rddmc_exitkernel_*); pass
    ``.buffer`` as ``run(surrogate=...)``.  ``windows`` lists each cloud's (i_lo, i_hi, j_lo, j_hi)."""

    def __init__(self, problem, min_steps: float = 64.0, tail: float = 1e-13, stream=None):
        import torch
        lib = load()
        b = problem.batch
        self.cfg = ExitKernelCfg_t(float(min_steps), float(tail))
        sb = C.c_size_t()
        _check(lib.rddmc_exitkernel_scratch_bytes(b.ref(), C.byref(sb)))
        scratch = torch.empty(max(int(sb.value), 256), dtype=torch.uint8, device=problem.tables.device)
        nbytes, nst = C.c_size_t(), C.c_uint64()
        win = np.zeros(4 * len(b.meds), dtype=np.int32)
        _check(lib.rddmc_exitkernel_bytes(b.ref(), C.c_void_p(problem.tables.data_ptr()), C.byref(self.cfg),
                                          C.c_void_p(scratch.data_ptr()), sb.value, C.byref(nbytes), C.byref(nst),
                                          win.ctypes.data, _stream(stream)))
        self.n_states = int(nst.value)
        self.windows = [tuple(int(v) for v in win[4 * c:4 * c + 4]) for c in range(len(b.meds))]
        self.buffer = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=problem.tables.device)
        _check(lib.rddmc_exitkernel_build(b.ref(), C.c_void_p(problem.tables.data_ptr()), C.byref(self.cfg),
                                          C.c_void_p(scratch.data_ptr()), sb.value,
                                          C.c_void_p(self.buffer.data_ptr()), nbytes.value, _stream(stream)))


class Problem:
    """Device buffers for one batch: tables, tallies and the work counter (torch tensors)."""

    def __init__(self, meds, keep_rates=False, device="cuda", stream=None, streams=None):
        import torch
        if isinstance(meds, _media.Medium):
            meds = [meds]
        self.batch = Batch(meds, keep_rates=keep_rates, streams=streams)
        self.stream = stream
        self.tables = torch.empty(table_bytes(self.batch), dtype=torch.uint8, device=device)
        self.tallies = torch.empty(tally_bytes(self.batch) // 8, dtype=torch.int64, device=device)
        self.work = torch.zeros(work_bytes(self.batch) // 8, dtype=torch.int64, device=device)
        build_leakage(self.batch, self.tables, stream)
        tally_reset(self.batch, self.tallies, stream)

    @property
    def total_packets(self):
        return sum(int(m.n_packets) for m in self.batch.meds)

    def reset(self):
        tally_reset(self.batch, self.tallies, self.stream)

    def run(self, **kw):
        transport(self.batch, self.tables, self.tallies, self.work, stream=self.stream, **kw)

    def capture(self, **kw):
        """Capture one rddmc_transport call (work-counter reset, lane walk, cooperative tail
        walk) into a HIP graph; ``graph.replay()`` re-runs it on the current stream, adding to
        the tallies.  The run parameters are fixed at capture time."""
        import torch
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            transport(self.batch, self.tables, self.tallies, self.work, stream=None, **kw)
        return g

    def results(self):
        return tally(self.batch, self.tallies, self.stream)

    def read_tables(self, cloud=0, want_rates=True):
        return read_tables(self.batch, self.tables, cloud, want_rates, self.stream)

    def read_redistribution(self, cloud=0):
        return read_redistribution(self.batch, self.tables, cloud, self.stream)


def mdn_bytes(max_batch):
    lib = load()
    pb, wb, npar = C.c_size_t(), C.c_size_t(), C.c_int64()
    _check(lib.rddmc_mdn_bytes(int(max_batch), C.byref(pb), C.byref(wb), C.byref(npar)))
    return pb.value, wb.value, npar.value


class Mdn:
    """Device buffers of the escape-surrogate network (parameters, optimiser state, work)."""

    def __init__(self, max_batch=4096, seed=0, device="cuda", stream=None):
        import torch
        self.max_batch = int(max_batch)
        pb, wb, self.n_params = mdn_bytes(self.max_batch)
        self.params = torch.zeros(pb // 4, dtype=torch.float32, device=device)
        self.work = torch.zeros(wb // 4 + 64, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.stream = stream
        self.step = 0
        _check(load().rddmc_mdn_init(C.c_void_p(self.params.data_ptr()), int(seed), _stream(stream)))

    def set_theta(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == self.n_params
        _check(load().rddmc_mdn_set(C.c_void_p(self.params.data_ptr()), th.ctypes.data, _stream(self.stream)))
        self.step = 0

    def get(self):
        th = np.zeros(self.n_params, dtype=np.float32)
        g = np.zeros(self.n_params, dtype=np.float32)
        _check(load().rddmc_mdn_get(C.c_void_p(self.params.data_ptr()), th.ctypes.data, g.ctypes.data,
                                    _stream(self.stream)))
        return th, g

    def forward(self, x):
        import torch
        n = int(x.shape[0])
        out = torch.empty((n, 128), dtype=torch.float32, device=x.device)
        _check(load().rddmc_mdn_forward(C.c_void_p(self.params.data_ptr()), C.c_void_p(self.work.data_ptr()),
                                        self.max_batch, C.c_void_p(x.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                        _stream(self.stream)))
        return out

    def loss_grad(self, x, y):
        n = int(x.shape[0])
        _check(load().rddmc_mdn_loss_grad(C.c_void_p(self.params.data_ptr()), C.c_void_p(self.work.data_ptr()),
                                          self.max_batch, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), n,
                                          C.c_void_p(self.loss.data_ptr()), _stream(self.stream)))
        return self.loss

    def adam(self, lr):
        self.step += 1
        _check(load().rddmc_mdn_adam(C.c_void_p(self.params.data_ptr()), self.step, float(lr), _stream(self.stream)))

    def train_step(self, x, y, lr):
        loss = self.loss_grad(x, y)
        self.adam(lr)
        return loss
