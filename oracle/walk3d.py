"""O1-3D wrapper: the literal FP64 hybrid DDMC / MC walker on Cartesian grids
(oracle/walk3d.c) -- test infrastructure only."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

from . import linemath
from . import tables as tb

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libo1walk3d.so")
TIME_BINS = 128
STEP_BINS = 64


def build_lib():
    src = os.path.join(HERE, "walk3d.c")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", LIB, src, "-lm", "-lpthread"])
    return LIB


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nb", C.c_int32),
                ("fx", C.c_void_p), ("fy", C.c_void_p), ("fz", C.c_void_p), ("edges", C.c_void_p),
                ("k", C.c_void_p), ("thick", C.c_void_p), ("rate_face", C.c_void_p),
                ("face_mc", C.c_void_p), ("rate_dn", C.c_void_p), ("rate_up", C.c_void_p),
                ("rho", C.c_void_p), ("shift", C.c_void_p), ("k0", C.c_void_p), ("a", C.c_void_p),
                ("T", C.c_void_p), ("u", C.c_void_p), ("lambda_", C.c_double), ("n_src", C.c_int32),
                ("src_state", C.c_void_p), ("src_pos", C.c_void_p), ("src_x", C.c_void_p),
                ("src_cdf", C.c_void_p), ("x_crit", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("spectrum", C.c_void_p), ("pixels", C.c_void_p), ("time_hist", C.c_void_p),
                ("step_hist", C.c_void_p), ("t_sum", C.c_double), ("t2_sum", C.c_double),
                ("steps_sum", C.c_double), ("mc_steps_sum", C.c_double), ("escaped", C.c_int64),
                ("capped", C.c_int64), ("to_mc", C.c_int64), ("to_ddmc", C.c_int64),
                ("reflected", C.c_int64), ("steps2_sum", C.c_double), ("mc_steps2_sum", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_lib()
        _lib = C.CDLL(LIB)
        _lib.o3_run.restype = C.c_int
        _lib.o3_run.argtypes = [C.POINTER(_Problem), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                                C.c_int, C.POINTER(_Result)]
        _lib.o3_dawson.restype = C.c_double
        _lib.o3_dawson.argtypes = [C.c_double]
        _lib.o3_voigt.restype = C.c_double
        _lib.o3_voigt.argtypes = [C.c_double, C.c_double]
        _lib.o3_upar_samples.restype = None
        _lib.o3_upar_samples.argtypes = [C.c_double, C.c_double, C.c_uint64, C.c_int64, C.c_void_p]
        _lib.o3_redistribution_samples.restype = None
        _lib.o3_redistribution_samples.argtypes = [C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                                   C.c_void_p]
    return _lib


def dawson(x):
    return _load().o3_dawson(float(x))


def voigt(a, x):
    return _load().o3_voigt(float(a), float(x))


def upar_samples(a, x, n, seed=1):
    out = np.zeros(int(n))
    _load().o3_upar_samples(float(a), float(x), int(seed), int(n), out.ctypes.data)
    return out


def redistribution_samples(a, x, n, seed=1, x_crit=0.0):
    """Outgoing comoving frequencies of n scatterings of a photon absorbed at x (optional
    core-skipping above x_crit)."""
    out = np.zeros(int(n))
    _load().o3_redistribution_samples(float(a), float(x), float(x_crit), int(seed), int(n), out.ctypes.data)
    return out


@dataclasses.dataclass
class Walk3DResult:
    spectrum: np.ndarray     # (6, nb+2)
    pixels: np.ndarray
    time_hist: np.ndarray
    step_hist: np.ndarray
    t_sum: float
    t2_sum: float
    steps_sum: float
    mc_steps_sum: float
    escaped: int
    capped: int
    to_mc: int
    to_ddmc: int
    reflected: int
    n_packets: int
    steps2_sum: float = 0.0
    mc_steps2_sum: float = 0.0

    @property
    def t_mean(self):
        return self.t_sum / max(self.escaped, 1)

    @property
    def steps_mean(self):
        return self.steps_sum / max(self.n_packets, 1)

    @property
    def steps_var(self):
        return self.steps2_sum / max(self.n_packets, 1) - self.steps_mean ** 2

    @property
    def mc_steps_mean(self):
        return self.mc_steps_sum / max(self.n_packets, 1)

    @property
    def mc_steps_var(self):
        return self.mc_steps2_sum / max(self.n_packets, 1) - self.mc_steps_mean ** 2

    @property
    def t_var(self):
        return self.t2_sum / max(self.escaped, 1) - self.t_mean ** 2


def run(m, n_packets=None, seed=0, first_id=0, max_steps=(1 << 62), n_threads=None, tabs=None):
    lib = _load()
    assert m.geometry == tb.CART3D
    t = tabs if tabs is not None else tb.build(m)
    nx, ny, nz = m.n_cells
    n = int(m.n_packets if n_packets is None else n_packets)
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    T = np.asarray(m.temp, dtype=np.float64)
    vth = linemath.v_thermal(T)
    vel = np.zeros((t.nc, 3)) if m.vel is None else np.asarray(m.vel, dtype=np.float64).reshape(t.nc, 3)
    u = vel / vth[:, None]
    src = tb.locate_sources(m)
    # one emission record per (source, state) with that source's position and frequency
    st, pos, xs, pr = [], [], [], []
    nsrc = len(m.src_x)
    for s in range(nsrc):
        one = m.replace(src_pos=np.asarray(m.src_pos)[s:s + 1], src_x=np.asarray(m.src_x)[s:s + 1])
        for state, p in tb.locate_sources(one):
            st.append(state)
            pos.append(np.asarray(m.src_pos)[s])
            xs.append(float(np.asarray(m.src_x)[s]))
            pr.append(p / nsrc)
    cdf = np.cumsum(pr)
    cdf[-1] = 1.0
    P = _Problem(nx, ny, nz, t.nb, arr(m.faces[0], np.float64), arr(m.faces[1], np.float64),
                 arr(m.faces[2], np.float64), arr(t.bin_edges, np.float64), arr(t.k, np.float64),
                 arr(t.thick, np.uint8), arr(t.rate_face, np.float64), arr(t.face_is_mc, np.uint8),
                 arr(t.rate_dn, np.float64), arr(t.rate_up, np.float64), arr(t.rho, np.float64),
                 arr(t.shift, np.float64), arr(m.k0, np.float64), arr(linemath.damping(T), np.float64),
                 arr(T, np.float64), arr(u, np.float64), float(m.lam), len(st), arr(st, np.int64),
                 arr(np.array(pos), np.float64), arr(xs, np.float64), arr(cdf, np.float64), float(m.x_crit))
    spec = np.zeros((6, t.nb + 2), dtype=np.int64)
    pix = np.zeros(2 * (ny * nz + nx * nz + nx * ny), dtype=np.int64)
    th = np.zeros(TIME_BINS + 2, dtype=np.int64)
    sh = np.zeros(STEP_BINS, dtype=np.int64)
    R = _Result(spec.ctypes.data, pix.ctypes.data, th.ctypes.data, sh.ctypes.data, 0.0, 0.0, 0.0, 0.0,
                0, 0, 0, 0, 0, 0.0, 0.0)
    rc = lib.o3_run(C.byref(P), first_id, n, seed, max_steps, n_threads or min(16, os.cpu_count() or 1), C.byref(R))
    if rc != 0:
        raise RuntimeError("o3_run failed")
    return Walk3DResult(spec, pix, th, sh, R.t_sum, R.t2_sum, R.steps_sum, R.mc_steps_sum, R.escaped,
                        R.capped, R.to_mc, R.to_ddmc, R.reflected, n, R.steps2_sum, R.mc_steps2_sum)
