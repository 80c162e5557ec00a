"""Learned escape surrogate: training data from the walk, training, and attaching.

The surrogate stands in for the DDMC walk of a packet inside one thick cell of a 1D cloud:
all the frequency steps (Sec. 2.3) until the first spatial leak become one exit (face,
exit frequency, time) drawn from a mixture-density network.  Everything numeric runs in
the HIP library: sub-walks (rddmc_surrogate_samples), the network's training on BF16
matrix cores (rddmc_mdn_*), and the per-state tables it is evaluated into
(rddmc_surrogate_attach).  This module builds the probe media the sub-walks run in and
drives the calls.

Probe media are three-cell slab or spherical-shell segments of a uniform medium whose
middle cell has the sampled parameters: optical width tau_c = k0 w, temperature (damping
a), bin width dx (uniform grid, both bin phases), Doppler shift s across each face from a
linear outflow, and shell index (face geometry).  Sub-walks start in the middle cell at a
bin whose centre lies within x_core of the line centre.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import media, rddmc

_A_1E4 = 4.702e-4
_VTH_1E4 = 12.85

# Training recipe: probe media, samples per probe (8192 x 12208 = 1.0e8 samples), epochs
# (Adam, cosine-decayed rate), the step budget above which a probe's samples come from the
# exact in-cell law instead of run sub-walks (about 38 % of the samples are run sub-walks).
TRAIN_PROBES = 8192
TRAIN_PER_PROBE = 12208
TRAIN_EPOCHS = 4
TRAIN_STEP_BUDGET = 2.0e5


@dataclasses.dataclass
class Domain:
    """The trained domain (the walk uses the network only inside it)."""
    tau_min: float = 1.0e5
    tau_max: float = 1.0e7
    a_min: float = 1.4e-4
    a_max: float = 5.0e-3
    dx_min: float = 0.2
    dx_max: float = 4.5
    shift_max: float = 0.5
    g_min: float = 0.75
    g_max: float = 1.3
    x_core: float = 3.0

    def cfg(self) -> rddmc.SurrogateCfg_t:
        return rddmc.SurrogateCfg_t(self.tau_min, self.tau_max, self.a_min, self.a_max, self.dx_min, self.dx_max,
                                    self.shift_max, self.g_min, self.g_max, self.x_core)


def train_domain() -> "Domain":
    """The trained domain: cell optical widths 1e4 .. 1e9, bins 0.5 .. 4.5 Doppler widths."""
    return Domain(tau_min=1.0e4, tau_max=1.0e9, dx_min=0.5, dx_max=4.5)


def use_domain() -> "Domain":
    """Where the walk uses the network: the trained domain above tau_c = 1e5."""
    return Domain(tau_min=1.0e5, tau_max=1.0e9, dx_min=0.5, dx_max=4.5)


def probe_medium(tau_c, a, dx, shift, shell, odd_bins, f_mu=0.5, lam=0.7104) -> media.Medium:
    """Three cells of unit width; cell 1 is the probed one.  shell = None: slab; else the
    segment spans radii [shell, shell + 3].  shift <= 0 is the eq. 20 shift of an outflow
    (neighbours recede)."""
    T = 1.0e4 * (_A_1E4 / a) ** 2
    vth = _VTH_1E4 * math.sqrt(T / 1.0e4)
    S = (a * tau_c) ** (1.0 / 3.0)
    x_max = max(10.0 * S + 12.0, 4.0 * dx)
    nb = 2 * int(math.ceil(x_max / dx)) + (1 if odd_bins else 0)
    half = 0.5 * nb * dx
    edges = media.uniform_edges(half, nb)
    dv = -shift * vth / f_mu
    vel = np.array([0.0, dv, 2.0 * dv])
    if shell is None:
        geom, faces = media.SLAB, np.array([-1.5, -0.5, 0.5, 1.5])
    else:
        geom, faces = media.SPHERE, float(shell) + np.arange(4, dtype=np.float64)
    return media.Medium(geometry=geom, n_cells=(3, 1, 1), faces=[faces, np.array([0.0, 1.0]), np.array([0.0, 1.0])],
                        bin_edges=edges, k0=np.full(3, float(tau_c)), temp=np.full(3, T), vel=vel,
                        src_pos=np.array([[0.5 * (faces[1] + faces[2]), 0.0, 0.0]]), src_x=np.array([0.0]),
                        n_packets=1, tau_threshold=0.0, f_mu=f_mu, lam=lam, name="probe")


def sample_probes(n, dom: Domain, seed=0, slab_fraction=0.2) -> List[media.Medium]:
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        tau = math.exp(rng.uniform(math.log(dom.tau_min), math.log(dom.tau_max)))
        a = math.exp(rng.uniform(math.log(dom.a_min), math.log(dom.a_max)))
        dx = math.exp(rng.uniform(math.log(dom.dx_min), math.log(dom.dx_max)))
        shift = -rng.uniform(0.0, dom.shift_max)
        shell = None if rng.random() < slab_fraction else float(round(math.exp(rng.uniform(math.log(8), math.log(600)))))
        out.append(probe_medium(tau, a, dx, shift, shell, odd_bins=bool(rng.integers(0, 2))))
    return out


def core_bins(m, x_core):
    e = np.asarray(m.bin_edges)
    c = 0.5 * (e[:-1] + e[1:])
    j = np.nonzero(np.abs(c) <= x_core)[0]
    if len(j) == 0:
        j = np.array([int(np.argmin(np.abs(c)))])
    return j


class Data:
    """Sub-walk samples on the device: X [n, 16], Y [n, 3] (rows with face -1 dropped)."""

    def __init__(self, x, y, steps):
        self.x, self.y, self.steps = x, y, steps

    @property
    def n(self):
        return int(self.x.shape[0])


def generate(probes, per_probe, dom: Domain, seed=0, max_steps=1 << 34, stream=None, bins=None) -> Data:
    """Run per_probe sub-walks from random core bins of every probe's middle cell (or from
    bins[i] of probe i).  Probes of each geometry run as one batch."""
    import torch
    geoms = sorted({m.geometry for m in probes})
    if len(geoms) > 1:
        parts = []
        for k, gm in enumerate(geoms):
            idx = [i for i, m in enumerate(probes) if m.geometry == gm]
            parts.append(generate([probes[i] for i in idx], per_probe, dom, seed + 7919 * k, max_steps, stream,
                                  None if bins is None else [bins[i] for i in idx]))
        return Data(torch.cat([d.x for d in parts]), torch.cat([d.y for d in parts]),
                    torch.cat([d.steps for d in parts]))
    rng = np.random.default_rng(seed + 1)
    batch = rddmc.Batch(probes)
    tables = torch.empty(rddmc.table_bytes(batch), dtype=torch.uint8, device="cuda")
    rddmc.build_leakage(batch, tables, stream)
    clouds, states = [], []
    for ci, m in enumerate(probes):
        js = core_bins(m, dom.x_core)
        pick = rng.choice(js, size=per_probe) if bins is None else np.full(per_probe, int(bins[ci]))
        clouds.append(np.full(per_probe, ci, dtype=np.int32))
        states.append((1 * m.n_bins + pick).astype(np.int32))
    hc = np.ascontiguousarray(np.concatenate(clouds))
    hs = np.ascontiguousarray(np.concatenate(states))
    n = len(hc)
    x = torch.empty((n, 16), dtype=torch.float32, device="cuda")
    y = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    st = torch.empty(n, dtype=torch.int64, device="cuda")
    scratch = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    lib = rddmc.load()
    rddmc._check(lib.rddmc_surrogate_samples(batch.ref(), rddmc.C.c_void_p(tables.data_ptr()), hc.ctypes.data,
                                             hs.ctypes.data, n, int(seed), int(max_steps),
                                             rddmc.C.c_void_p(scratch.data_ptr()), 8 * n,
                                             rddmc.C.c_void_p(x.data_ptr()), rddmc.C.c_void_p(y.data_ptr()),
                                             rddmc.C.c_void_p(st.data_ptr()), rddmc._stream(stream)))
    keep = y[:, 0] >= 0
    return Data(x[keep].contiguous(), y[keep].contiguous(), st[keep].contiguous())


def generate_exact(probes, per_probe, dom: Domain, seed=0, bins_per_probe=8, pairs_per_call=2048,
                   bins=None) -> Data:
    """Samples of the probes' middle-cell exits drawn from the exact in-cell law
    (rddmc_exitlaw_samples): per probe, per_probe samples spread over bins_per_probe random
    core bins (or all from bins[i] of probe i).  Same layout as generate()."""
    import torch
    geoms = sorted({m.geometry for m in probes})
    if len(geoms) > 1:
        parts = [generate_exact([m for m in probes if m.geometry == gm], per_probe, dom, seed + 7919 * k,
                                bins_per_probe, pairs_per_call,
                                None if bins is None else [b for m, b in zip(probes, bins) if m.geometry == gm])
                 for k, gm in enumerate(geoms)]
        return Data(torch.cat([d.x for d in parts]), torch.cat([d.y for d in parts]),
                    torch.cat([d.steps for d in parts]))
    rng = np.random.default_rng(seed + 3)
    batch = rddmc.Batch(probes)
    tables = torch.empty(rddmc.table_bytes(batch), dtype=torch.uint8, device="cuda")
    rddmc.build_leakage(batch, tables)
    pc, ps, cnt = [], [], []
    for ci, m in enumerate(probes):
        js = core_bins(m, dom.x_core)
        if bins is not None:
            pick = np.array([int(bins[ci])])
        else:
            pick = rng.choice(js, size=min(bins_per_probe, len(js)), replace=len(js) < bins_per_probe)
        share = np.full(len(pick), per_probe // len(pick))
        share[:per_probe - share.sum()] += 1
        for j, k in zip(pick, share):
            pc.append(ci)
            ps.append(m.n_bins + int(j))
            cnt.append(int(k))
    pc, ps, cnt = (np.ascontiguousarray(np.array(v, dtype=np.int32)) for v in (pc, ps, cnt))
    nb_max = max(m.n_bins for m in probes)
    lib = rddmc.load()
    xs, ys = [], []
    for a in range(0, len(pc), pairs_per_call):
        b = min(len(pc), a + pairs_per_call)
        n = b - a
        rows = int(cnt[a:b].sum())
        x = torch.empty((rows, 16), dtype=torch.float32, device="cuda")
        y = torch.empty((rows, 3), dtype=torch.float32, device="cuda")
        scr = torch.empty(6 * 256 + 20 * n + 88 * nb_max * n, dtype=torch.uint8, device="cuda")
        ca, sa, na = (np.ascontiguousarray(v[a:b]) for v in (pc, ps, cnt))
        rddmc._check(lib.rddmc_exitlaw_samples(batch.ref(), rddmc.C.c_void_p(tables.data_ptr()), ca.ctypes.data,
                                               sa.ctypes.data, na.ctypes.data, n, int(seed) * 7 + a,
                                               rddmc.C.c_void_p(scr.data_ptr()), scr.numel(),
                                               rddmc.C.c_void_p(x.data_ptr()), rddmc.C.c_void_p(y.data_ptr()),
                                               None))
        xs.append(x)
        ys.append(y)
    x = torch.cat(xs)
    y = torch.cat(ys)
    return Data(x, y, torch.zeros(x.shape[0], dtype=torch.int64, device="cuda"))


def expected_subwalk(m) -> float:
    """Rough length of a middle-cell sub-walk of a probe, 0.6 tau_c / dx^2 steps (the scaling
    measured on the sub-walk data): the split between run sub-walks and exact-law draws."""
    e = np.asarray(m.bin_edges)
    return 0.6 * float(m.k0[1]) * float(m.faces[0][2] - m.faces[0][1]) / float(e[1] - e[0]) ** 2


def generate_mixed(probes, per_probe, dom: Domain, seed=0, step_budget=2.0e6, max_steps=1 << 30) -> Data:
    """Training data over a wide domain: probes whose sub-walks are expected to take at most
    step_budget steps run them (generate); the rest draw from the exact in-cell law."""
    import torch
    short = [m for m in probes if expected_subwalk(m) <= step_budget]
    long = [m for m in probes if expected_subwalk(m) > step_budget]
    parts = []
    if short:
        parts.append(generate(short, per_probe, dom, seed=seed, max_steps=max_steps))
    if long:
        parts.append(generate_exact(long, per_probe, dom, seed=seed + 1))
    return Data(torch.cat([d.x for d in parts]), torch.cat([d.y for d in parts]),
                torch.cat([d.steps for d in parts]))


def train(net: rddmc.Mdn, data: Data, epochs=30, batch=4096, lr=2e-3, lr_final=2e-4, seed=0, log=None):
    """Adam on shuffled minibatches (cosine-decayed learning rate); returns the per-epoch
    mean training loss."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = data.n
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        acc = torch.zeros(1, device="cuda")
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            xb = data.x[idx].contiguous()
            yb = data.y[idx].contiguous()
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / max(total - 1, 1)))
            acc += net.train_step(xb, yb, rate)
            k += 1
        hist.append(float(acc.cpu()[0]) / steps_per_epoch)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def mean_nll(net: rddmc.Mdn, data: Data, batch=4096) -> float:
    """Mean negative log-likelihood of the network over a data set (in minibatches; the
    parameters are left unchanged, the gradient slot is overwritten)."""
    import torch
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    for a in range(0, data.n, batch):
        b = min(data.n, a + batch)
        acc += net.loss_grad(data.x[a:b].contiguous(), data.y[a:b].contiguous()).double() * (b - a)
    return float(acc.cpu()[0]) / max(data.n, 1)


class Attached:
    """Per-state sampling records of a batch (pass .buffer as the transport's surrogate)."""

    def __init__(self, problem, net: rddmc.Mdn, dom: Domain, stream=None):
        import torch
        lib = rddmc.load()
        self.cfg = dom.cfg()
        b = problem.batch
        nbytes = rddmc.C.c_size_t()
        nst = rddmc.C.c_uint64()
        rddmc._check(lib.rddmc_surrogate_bytes(b.ref(), rddmc.C.byref(self.cfg), net.max_batch,
                                               rddmc.C.byref(nbytes), rddmc.C.byref(nst)))
        self.n_states = nst.value
        self.buffer = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        rddmc._check(lib.rddmc_surrogate_attach(b.ref(), rddmc.C.c_void_p(problem.tables.data_ptr()),
                                                rddmc.C.c_void_p(net.params.data_ptr()),
                                                rddmc.C.c_void_p(net.work.data_ptr()), net.max_batch,
                                                rddmc.C.byref(self.cfg), rddmc.C.c_void_p(self.buffer.data_ptr()),
                                                nbytes.value, rddmc._stream(stream)))
        self.windows = []
        for c in range(len(b.meds)):
            w = np.zeros(4, dtype=np.int32)
            rddmc._check(lib.rddmc_surrogate_window(b.ref(), rddmc.C.byref(self.cfg), c, w.ctypes.data))
            self.windows.append(tuple(int(v) for v in w))


def window(med, dom: Domain):
    """Host query of one cloud's window (i_lo, i_hi, j_lo, j_hi)."""
    lib = rddmc.load()
    b = rddmc.Batch([med])
    cfg = dom.cfg()
    w = np.zeros(4, dtype=np.int32)
    rddmc._check(lib.rddmc_surrogate_window(b.ref(), rddmc.C.byref(cfg), 0, w.ctypes.data))
    return tuple(int(v) for v in w)
