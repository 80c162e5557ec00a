"""O1 wrapper: the literal FP64 C walker (oracle/walk.c) -- test infrastructure only.

``run(medium, n_packets, seed)`` builds the oracle's own FP64 tables
(oracle/tables.py), hands them to the C walker and returns plain numpy tallies.
The shared library is compiled from oracle/walk.c by ``build_lib()`` (gcc).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

from . import tables as tb

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libo1walk.so")
TIME_BINS = 128
STEP_BINS = 64


def build_lib():
    src = os.path.join(HERE, "walk.c")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", LIB, src, "-lm",
                           "-lpthread"])
    return LIB


class _Problem(C.Structure):
    _fields_ = [("nc", C.c_int32), ("nb", C.c_int32), ("nf", C.c_int32), ("moving", C.c_int32),
                ("rate_face", C.c_void_p), ("rate_dn", C.c_void_p), ("rate_up", C.c_void_p),
                ("nbr", C.c_void_p), ("rho", C.c_void_p), ("shift", C.c_void_p),
                ("u_n", C.c_void_p), ("edges", C.c_void_p), ("n_src", C.c_int32),
                ("src_state", C.c_void_p), ("src_cdf", C.c_void_p), ("n_rows", C.c_int32),
                ("face_row", C.c_void_p)]


class _Result(C.Structure):
    _fields_ = [("spectrum", C.c_void_p), ("time_hist", C.c_void_p), ("step_hist", C.c_void_p),
                ("t_sum", C.c_double), ("t2_sum", C.c_double), ("steps_sum", C.c_double),
                ("steps2_sum", C.c_double), ("escaped", C.c_int64), ("capped", C.c_int64),
                ("steps_max", C.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_lib()
        _lib = C.CDLL(LIB)
        _lib.o1_run.restype = C.c_int
        _lib.o1_run.argtypes = [C.POINTER(_Problem), C.c_uint64, C.c_uint64, C.c_uint64,
                                C.c_uint64, C.c_int, C.POINTER(_Result)]
    return _lib


@dataclasses.dataclass
class WalkResult:
    spectrum: np.ndarray     # (rows, nb+2) int64 counts
    faces: list
    time_hist: np.ndarray
    step_hist: np.ndarray
    t_sum: float
    t2_sum: float
    steps_sum: float
    steps2_sum: float
    escaped: int
    capped: int
    steps_max: int
    n_packets: int

    @property
    def t_mean(self):
        return self.t_sum / max(self.escaped, 1)

    @property
    def steps_mean(self):
        return self.steps_sum / max(self.n_packets, 1)


def run(m, n_packets=None, seed=0, first_id=0, max_steps=(1 << 62), n_threads=None, tabs=None):
    lib = _load()
    t = tabs if tabs is not None else tb.build(m)
    if not np.all(t.thick):
        raise ValueError("this walker covers pure DDMC (all states thick)")
    n = int(m.n_packets if n_packets is None else n_packets)
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    esc_faces = sorted({f for f in range(t.nf) if np.any(t.nbr[:, f] == tb.NBR_VACUUM)})
    face_row = np.full(t.nf, -1, dtype=np.int32)
    for i, f in enumerate(esc_faces):
        face_row[f] = i
    src = tb.locate_sources(m)
    st = np.array([s for s, _ in src], dtype=np.int64)
    cdf = np.cumsum([p for _, p in src])
    cdf[-1] = 1.0
    P = _Problem(t.nc, t.nb, t.nf, int(t.moving), arr(t.rate_face, np.float64),
                 arr(t.rate_dn, np.float64), arr(t.rate_up, np.float64), arr(t.nbr, np.int64),
                 arr(t.rho, np.float64), arr(t.shift, np.float64), arr(t.u_n, np.float64),
                 arr(t.bin_edges, np.float64), len(st), arr(st, np.int64), arr(cdf, np.float64),
                 len(esc_faces), arr(face_row, np.int32))
    spec = np.zeros((len(esc_faces), t.nb + 2), dtype=np.int64)
    th = np.zeros(TIME_BINS + 2, dtype=np.int64)
    sh = np.zeros(STEP_BINS, dtype=np.int64)
    R = _Result(spec.ctypes.data, th.ctypes.data, sh.ctypes.data, 0.0, 0.0, 0.0, 0.0, 0, 0, 0)
    nthr = n_threads or min(16, os.cpu_count() or 1)   # at most 16 threads
    rc = lib.o1_run(C.byref(P), first_id, n, seed, max_steps, nthr, C.byref(R))
    if rc != 0:
        raise RuntimeError("o1_run failed")
    return WalkResult(spectrum=spec, faces=esc_faces, time_hist=th, step_hist=sh, t_sum=R.t_sum,
                      t2_sum=R.t2_sum, steps_sum=R.steps_sum, steps2_sum=R.steps2_sum,
                      escaped=R.escaped, capped=R.capped, steps_max=R.steps_max, n_packets=n)
