"""O1-1DH wrapper: the literal FP64 hybrid DDMC / continuous-MC walker on slabs and spherical
shells (oracle/walk1dh.c) -- test infrastructure only."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

from . import linemath
from . import tables as tb

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libo1walk1dh.so")
TIME_BINS = 128
STEP_BINS = 64
GROUP_FLAG = 1 << 2     # a cloud's flag bit: thin states use frequency groups (Sec. 5.3)
DUST_WEIGHT_FLAG = 1 << 3   # a cloud's flag bit: dust absorption by continuous weights (Sec. 2.4)


def build_lib():
    src = os.path.join(HERE, "walk1dh.c")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", LIB, src, "-lm", "-lpthread"])
    return LIB


class _Problem(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("nc", C.c_int32), ("nb", C.c_int32), ("faces", C.c_void_p),
                ("edges", C.c_void_p), ("k", C.c_void_p), ("thick", C.c_void_p), ("rate_face", C.c_void_p),
                ("face_mc", C.c_void_p), ("rate_dn", C.c_void_p), ("rate_up", C.c_void_p), ("nbr", C.c_void_p),
                ("rho", C.c_void_p), ("shift", C.c_void_p), ("k0", C.c_void_p), ("a", C.c_void_p),
                ("T", C.c_void_p), ("u", C.c_void_p), ("lambda_", C.c_double), ("x_crit", C.c_double),
                ("n_src", C.c_int32), ("src_state", C.c_void_p), ("src_pos", C.c_void_p), ("src_x", C.c_void_p),
                ("src_cdf", C.c_void_p), ("k_abs", C.c_void_p), ("k_sca", C.c_void_p), ("src_t", C.c_void_p),
                ("n_census", C.c_int32), ("census", C.c_void_p), ("group", C.c_int32), ("dust_weight", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("spectrum", C.c_void_p), ("time_hist", C.c_void_p), ("step_hist", C.c_void_p),
                ("t_sum", C.c_double), ("t2_sum", C.c_double), ("steps_sum", C.c_double),
                ("mc_steps_sum", C.c_double), ("steps2_sum", C.c_double), ("escaped", C.c_int64),
                ("capped", C.c_int64), ("to_mc", C.c_int64), ("to_ddmc", C.c_int64), ("reflected", C.c_int64),
                ("absorbed", C.c_int64), ("e_bin", C.c_void_p), ("e_path", C.c_void_p), ("e_accel", C.c_void_p),
                ("wspec", C.c_void_p), ("wspec2", C.c_void_p), ("wt_sum", C.c_double), ("wt2_sum", C.c_double),
                ("w_sum", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_lib()
        _lib = C.CDLL(LIB)
        _lib.oh_run.restype = C.c_int
        _lib.oh_run.argtypes = [C.POINTER(_Problem), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                                C.c_int, C.POINTER(_Result)]
    return _lib


@dataclasses.dataclass
class Walk1DHResult:
    spectrum: np.ndarray     # (rows, nb+2): slab rows = faces 0/1, sphere one row
    time_hist: np.ndarray
    step_hist: np.ndarray
    t_sum: float
    t2_sum: float
    steps_sum: float
    mc_steps_sum: float
    steps2_sum: float
    escaped: int
    capped: int
    to_mc: int
    to_ddmc: int
    reflected: int
    n_packets: int
    absorbed: int = 0
    e_bin: np.ndarray = None   # (n_census+1, nc, nb) packets in each state at each census time
    e_path: np.ndarray = None  # (n_census, nc, nb) residence time per census interval
    e_accel: np.ndarray = None  # (n_census, nc) eq. 18 optical-depth sums (z or r component)
    wspec: np.ndarray = None   # (rows, nb+2) escaped weight (continuous dust weights)
    wspec2: np.ndarray = None  # (rows, nb+2) escaped squared weight
    w_sum: float = 0.0
    wt_sum: float = 0.0
    wt2_sum: float = 0.0

    @property
    def t_mean_w(self):
        return self.wt_sum / self.w_sum if self.w_sum > 0 else 0.0

    @property
    def t_var_w(self):
        return self.wt2_sum / self.w_sum - self.t_mean_w ** 2 if self.w_sum > 0 else 0.0

    @property
    def t_mean(self):
        return self.t_sum / max(self.escaped, 1)

    @property
    def t_var(self):
        return self.t2_sum / max(self.escaped, 1) - self.t_mean ** 2

    @property
    def steps_mean(self):
        return self.steps_sum / max(self.n_packets, 1)

    @property
    def steps_var(self):
        return self.steps2_sum / max(self.n_packets, 1) - self.steps_mean ** 2


def run(m, n_packets=None, seed=0, first_id=0, max_steps=(1 << 62), n_threads=None, tabs=None, x_crit=None):
    """Walk ``n_packets`` packets of the 1D medium ``m`` (slab or sphere, pure or hybrid); the
    core-skipping threshold is the medium's unless ``x_crit`` is given."""
    lib = _load()
    if x_crit is None:
        x_crit = getattr(m, "x_crit", 0.0)
    assert m.geometry in (tb.SLAB, tb.SPHERE)
    t = tabs if tabs is not None else tb.build(m)
    n = int(m.n_packets if n_packets is None else n_packets)
    group = bool(int(m.flags) & GROUP_FLAG)
    weighted = bool(int(m.flags) & DUST_WEIGHT_FLAG)
    if weighted:
        assert m.dust_abs is not None
    if group:   # frequency groups (Sec. 5.3): static, isothermal clouds
        assert m.vel is None and np.all(np.asarray(m.temp) == np.asarray(m.temp).flat[0])
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    T = np.asarray(m.temp, dtype=np.float64)
    vth = linemath.v_thermal(T)
    vel = np.zeros(t.nc) if m.vel is None else np.asarray(m.vel, dtype=np.float64).reshape(t.nc)
    st, pos, xs, pr, tw = [], [], [], [], []
    nsrc = len(m.src_x)
    for s in range(nsrc):
        one = m.replace(src_pos=np.asarray(m.src_pos)[s:s + 1], src_x=np.asarray(m.src_x)[s:s + 1])
        for state, p in tb.locate_sources(one):
            st.append(state)
            pos.append(float(np.asarray(m.src_pos)[s][0]))
            xs.append(float(np.asarray(m.src_x)[s]))
            pr.append(p / nsrc)
            if m.src_t is not None:
                tw.extend(float(v) for v in np.asarray(m.src_t, dtype=np.float64).reshape(nsrc, 2)[s])
    cdf = np.cumsum(pr)
    cdf[-1] = 1.0
    P = _Problem(int(m.geometry), t.nc, t.nb, arr(m.faces[0], np.float64), arr(t.bin_edges, np.float64),
                 arr(t.k, np.float64), arr(t.thick, np.uint8), arr(t.rate_face, np.float64),
                 arr(t.face_is_mc, np.uint8), arr(t.rate_dn, np.float64), arr(t.rate_up, np.float64),
                 arr(t.nbr, np.int64), arr(t.rho, np.float64), arr(t.shift, np.float64), arr(m.k0, np.float64),
                 arr(linemath.damping(T), np.float64), arr(T, np.float64), arr(vel / vth, np.float64),
                 float(m.lam), float(x_crit), len(st), arr(st, np.int64), arr(pos, np.float64),
                 arr(xs, np.float64), arr(cdf, np.float64),
                 arr(m.dust_abs, np.float64) if m.dust_abs is not None else None,
                 arr(m.dust_sca, np.float64) if m.dust_sca is not None else None,
                 arr(tw, np.float64) if m.src_t is not None else None,
                 0 if m.census is None else len(m.census) - 1,
                 arr(m.census, np.float64) if m.census is not None else None, int(group), int(weighted))
    rows = 2 if m.geometry == tb.SLAB else 1
    spec = np.zeros((rows, t.nb + 2), dtype=np.int64)
    th = np.zeros(TIME_BINS + 2, dtype=np.int64)
    sh = np.zeros(STEP_BINS, dtype=np.int64)
    nce = 0 if m.census is None else len(m.census) - 1
    e_bin = np.zeros((nce + 1, t.nc, t.nb)) if nce else None
    e_path = np.zeros((nce, t.nc, t.nb)) if nce else None
    e_accel = np.zeros((nce, t.nc)) if nce else None
    wspec = np.zeros((rows, t.nb + 2)) if weighted else None
    wspec2 = np.zeros((rows, t.nb + 2)) if weighted else None
    R = _Result(spec.ctypes.data, th.ctypes.data, sh.ctypes.data, 0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0, 0, 0,
                e_bin.ctypes.data if nce else None, e_path.ctypes.data if nce else None,
                e_accel.ctypes.data if nce else None, wspec.ctypes.data if weighted else None,
                wspec2.ctypes.data if weighted else None, 0.0, 0.0, 0.0)
    rc = lib.oh_run(C.byref(P), first_id, n, seed, max_steps, n_threads or min(16, os.cpu_count() or 1), C.byref(R))
    if rc != 0:
        raise RuntimeError("oh_run failed")
    return Walk1DHResult(spec, th, sh, R.t_sum, R.t2_sum, R.steps_sum, R.mc_steps_sum, R.steps2_sum, R.escaped,
                         R.capped, R.to_mc, R.to_ddmc, R.reflected, n, R.absorbed, e_bin, e_path, e_accel,
                         wspec, wspec2, R.w_sum, R.wt_sum, R.wt2_sum)
