"""Seeded synthetic media and sources for rDDMC Lyman-alpha transfer.

This module only *describes* problems: grids, per-cell line-centre opacity,
temperature, bulk velocity, sources and packet counts.  It contains none of
the transport arithmetic (no Voigt profile, no leakage coefficients, no
random walk); both the GPU library and the CPU oracle read the same
``Medium`` objects produced here.

Units
-----
* Lengths are in units of the slab half-width / sphere radius ``R`` (slab,
  sphere) or of one cell width (Cartesian cube).  ``k0`` is therefore the
  line-centre optical depth per unit length, and the line-centre optical
  depth from the centre to the edge is ``tau0 = k0 * R`` (the paper's
  convention in its grey and resonant test problems, Sec. 3).
* Times are in units of ``length / c``.
* Frequencies are the dimensionless comoving ``x = (nu - nu0) / dnu_D`` of
  each cell (Doppler units of the cell's own temperature, Sec. 2.1).
* Velocities are in km/s.

Geometry codes: 0 = slab (1D Cartesian), 1 = sphere (radial shells),
2 = 3D Cartesian.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

SLAB, SPHERE, CART3D = 0, 1, 2

# Flags shared by both sides (the meanings are documented in include/rddmc.h).
FLAG_DIRICHLET = 1 << 0   # vacuum face uses a zero-intensity face instead of the extrapolation distance

# Lyman-alpha damping parameter at 1e4 K (Sec. 2.1); used here only to size
# the frequency range of a grid, never for transport.
_A_1E4 = 4.702e-4
_VTH_1E4 = 12.85  # km/s


def _a_of_T(T: float) -> float:
    return _A_1E4 / math.sqrt(T / 1.0e4)


def _vth_of_T(T: float) -> float:
    return _VTH_1E4 * math.sqrt(T / 1.0e4)


@dataclasses.dataclass
class Medium:
    geometry: int
    n_cells: tuple                 # (n0, n1, n2); 1D geometries use (n, 1, 1)
    faces: List[np.ndarray]        # per axis, n+1 increasing face coordinates
    bin_edges: np.ndarray          # n_bins+1 increasing comoving x edges
    k0: np.ndarray                 # per cell line-centre opacity [1/length]
    temp: np.ndarray               # per cell temperature [K]
    vel: Optional[np.ndarray]      # slab: v_z per cell; sphere: v_r per shell; cart: (n,3); None = static
    src_pos: np.ndarray            # (n_src, 3) source positions (slab: z; sphere: r; cart: x,y,z)
    src_x: np.ndarray              # (n_src,) source comoving frequencies
    n_packets: int
    tau_threshold: float = 0.0     # 0 = pure DDMC; otherwise >= 2
    f_mu: float = 0.5
    lam: float = 0.7104
    flags: int = 0
    name: str = ""
    x_crit: float = 0.0            # continuous-MC core-skipping threshold (0 = off)
    dust_abs: Optional[np.ndarray] = None   # per cell dust absorption coefficient [1/length]
    dust_sca: Optional[np.ndarray] = None   # per cell dust scattering coefficient [1/length]
    src_t: Optional[np.ndarray] = None      # (n_src, 2) emission windows [t_start, t_end]; None = flash at 0
    census: Optional[np.ndarray] = None     # census times (n+1 increasing edges) of the energy-density
                                            # estimators; None = no time-dependent tallies

    @property
    def n_bins(self) -> int:
        return int(len(self.bin_edges) - 1)

    @property
    def n_cells_total(self) -> int:
        return int(self.n_cells[0] * self.n_cells[1] * self.n_cells[2])

    def with_packets(self, n: int) -> "Medium":
        return dataclasses.replace(self, n_packets=int(n))

    def replace(self, **kw) -> "Medium":
        return dataclasses.replace(self, **kw)


GROUP_MC = 1 << 2      # Medium.flags bit: thin states use frequency groups (Sec. 5.3 eq. 42)
ALL_THIN = 1.0e300     # a tau_threshold above every state's optical width: no DDMC states
DUST_WEIGHT = 1 << 3   # Medium.flags bit: dust absorption by continuous packet weights (Sec. 2.4)


def uniform_edges(x_max: float, n_bins: int) -> np.ndarray:
    """n_bins+1 edges over [-x_max, x_max], exactly antisymmetric, with an exact 0 edge
    whenever n_bins is even."""
    i = np.arange(n_bins + 1, dtype=np.float64)
    return (2.0 * i - n_bins) / n_bins * x_max


def core_wing_crossover(a: float) -> float:
    """x_cw, where the Doppler core exp(-x^2) meets the damping wing a / (sqrt(pi) x^2)
    (Sec. 2.1): the root above 1 of x^2 - 2 ln x = ln(sqrt(pi) / a), by Newton's method."""
    rhs = math.log(math.sqrt(math.pi) / a)
    if rhs <= 1.0:
        raise ValueError(f"damping a = {a} leaves no core: x^2 - 2 ln x >= 1 for every x")
    x = max(1.5, math.sqrt(rhs + 2.0 * math.log(max(rhs, 1.0))))
    for _ in range(60):
        f = x * x - 2.0 * math.log(x) - rhs
        x_new = x - f / (2.0 * x - 2.0 / x)
        if abs(x_new - x) < 1e-15 * x:
            return x_new
        x = x_new
    return x


def efficient_edges(a: float, tau0: float, dz_over_R: float, x_max: Optional[float] = None,
                    dx_wing: Optional[float] = None) -> np.ndarray:
    """The frequency grid the paper recommends for pure rDDMC (Secs. 4.2 and 5.1): one central
    bin at least 2 x_cw wide (binning skips the core's complete redistribution; it takes
    max(2 x_cw, dx_wing)), wing bins of width dx_wing, an odd number of bins in all, over
    |x| <= x_max.

    dx_wing defaults to the width that matches the cell size by eq. 37,
    dx^3 / (a tau0) = 2.5 (dz / R)^2, and never goes below 1 (the Fokker-Planck treatment of
    the wings needs bins wider than the redistribution step); x_max defaults to
    2.5 (a tau0)^(1/3).  The outermost wing bins end at or just beyond x_max."""
    atau = a * tau0
    if x_max is None:
        x_max = 2.5 * atau ** (1.0 / 3.0)
    if dx_wing is None:
        dx_wing = max(1.0, (2.5 * atau * dz_over_R ** 2) ** (1.0 / 3.0))
    h = max(core_wing_crossover(a), 0.5 * dx_wing)
    if x_max <= h:
        raise ValueError(f"x_max = {x_max} lies inside the central bin (x_cw = {h})")
    n_w = int(math.ceil((x_max - h) / dx_wing - 1e-12))
    wing = h + dx_wing * np.arange(n_w + 1, dtype=np.float64)
    return np.concatenate([-wing[::-1], wing])


def slab(tau0: float, T: float, n_cells: int, n_bins: int, x_max: Optional[float] = None,
         x_max_factor: float = 6.0, n_packets: int = 1 << 16, tau_threshold: float = 0.0,
         src_z: float = 0.0, src_x: float = 0.0, vel: Optional[np.ndarray] = None,
         lam: float = 0.7104, flags: int = 0, name: str = "slab") -> Medium:
    """Uniform isothermal slab z in [-1, 1] with line-centre depth tau0 from centre to edge."""
    if x_max is None:
        x_max = x_max_factor * (_a_of_T(T) * tau0) ** (1.0 / 3.0)
    faces = [uniform_edges(1.0, n_cells), np.array([0.0, 1.0]), np.array([0.0, 1.0])]
    return Medium(geometry=SLAB, n_cells=(n_cells, 1, 1), faces=faces,
                  bin_edges=uniform_edges(x_max, n_bins),
                  k0=np.full(n_cells, float(tau0)), temp=np.full(n_cells, float(T)),
                  vel=None if vel is None else np.asarray(vel, dtype=np.float64),
                  src_pos=np.array([[src_z, 0.0, 0.0]]), src_x=np.array([src_x]),
                  n_packets=int(n_packets), tau_threshold=float(tau_threshold), lam=lam,
                  flags=flags, name=name)


def sphere(tau0: float, T: float, n_shells: int, n_bins: int, x_max: Optional[float] = None,
           x_max_factor: float = 6.0, n_packets: int = 1 << 22, tau_threshold: float = 0.0,
           v_max: float = 0.0, src_x: float = 0.0, lam: float = 0.7104, flags: int = 0,
           name: str = "sphere") -> Medium:
    """Uniform isothermal sphere r in [0, 1], central point source, optional Hubble-like
    outflow v(r) = v_max r / R evaluated at shell mid-radius."""
    if x_max is None:
        x_max = x_max_factor * (_a_of_T(T) * tau0) ** (1.0 / 3.0)
    r = np.linspace(0.0, 1.0, n_shells + 1)
    vel = None
    if v_max != 0.0:
        vel = v_max * 0.5 * (r[1:] + r[:-1])
    faces = [r, np.array([0.0, 1.0]), np.array([0.0, 1.0])]
    return Medium(geometry=SPHERE, n_cells=(n_shells, 1, 1), faces=faces,
                  bin_edges=uniform_edges(x_max, n_bins),
                  k0=np.full(n_shells, float(tau0)), temp=np.full(n_shells, float(T)), vel=vel,
                  src_pos=np.array([[0.0, 0.0, 0.0]]), src_x=np.array([src_x]),
                  n_packets=int(n_packets), tau_threshold=float(tau_threshold), lam=lam,
                  flags=flags, name=name)


# --------------------------------------------------------------------------------------
# The workloads.  Sizes follow the problem statements; derived ranges are documented where
# the statement leaves them open.
# --------------------------------------------------------------------------------------

def config_slab(n_packets: int = 1 << 16) -> Medium:
    """Static uniform slab: tau0 = 1e5, T = 1e4 K, 64 cells x 128 bins over
    |x| <= 6 (a tau0)^(1/3), monochromatic source at z = 0, x = 0."""
    return slab(1.0e5, 1.0e4, 64, 128, n_packets=n_packets, name="slab_tau1e5_64x128")


def config_sphere(n_packets: int = 1 << 22) -> Medium:
    """Static uniform sphere: tau0 = 1e7, T = 1e4 K, 256 shells x 512 bins over
    |x| <= 6 (a tau0)^(1/3), central point source at x = 0."""
    return sphere(1.0e7, 1.0e4, 256, 512, n_packets=n_packets, name="sphere_tau1e7_256x512")


def validation_slab(n_packets: int = 1 << 20) -> Medium:
    """The paper's converged slab test: a tau0 = 1e9 at T = 10 K, 201 cells x 101 bins
    over |x| <= 2.5 (a tau0)^(1/3) (odd counts so the source sits in a cell/bin centre)."""
    T = 10.0
    a = _a_of_T(T)
    tau0 = 1.0e9 / a
    return slab(tau0, T, 201, 101, x_max=2.5 * 1.0e3, n_packets=n_packets, name="vslab_atau1e9")


def validation_sphere(n_packets: int = 1 << 20) -> Medium:
    T = 10.0
    a = _a_of_T(T)
    tau0 = 1.0e9 / a
    return sphere(tau0, T, 200, 201, x_max=2.5 * 1.0e3, n_packets=n_packets, name="vsphere_atau1e9")


@dataclasses.dataclass
class SweepCloud:
    tau0: float
    T: float
    n_shells: int
    n_bins: int
    v_max: float
    n_packets: int


def sweep_parameters(n_clouds: int = 256, seed: int = 3) -> List[SweepCloud]:
    """Cloud parameters of the batched sweep, drawn with PCG64(seed) in a fixed order:
    tau0 = 10^U(4,9), T = 10^U(2,5) K, shells ~ U{32..512}, bins ~ U{256..1024},
    v_max ~ U(0, 200) km/s, packets = round(2^U(14,18))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_clouds):
        tau0 = 10.0 ** rng.uniform(4.0, 9.0)
        T = 10.0 ** rng.uniform(2.0, 5.0)
        ns = int(rng.integers(32, 513))
        nb = int(rng.integers(256, 1025))
        vmax = float(rng.uniform(0.0, 200.0))
        npk = int(round(2.0 ** rng.uniform(14.0, 18.0)))
        out.append(SweepCloud(tau0, T, ns, nb, vmax, npk))
    return out


def sweep_cloud_medium(c: SweepCloud, tau_threshold: float = 0.0) -> Medium:
    """One sweep cloud: |x| <= 6 (a tau0)^(1/3) + 1.2 u_max with u_max = v_max / v_th."""
    u_max = c.v_max / _vth_of_T(c.T)
    x_max = 6.0 * (_a_of_T(c.T) * c.tau0) ** (1.0 / 3.0) + 1.2 * u_max
    return sphere(c.tau0, c.T, c.n_shells, c.n_bins, x_max=x_max, v_max=c.v_max,
                  n_packets=c.n_packets, tau_threshold=tau_threshold,
                  name=f"sweep_tau{c.tau0:.3g}_T{c.T:.3g}")


def config_sweep(n_clouds: int = 256, seed: int = 3, packet_scale: float = 1.0,
                 tau_threshold: float = 0.0) -> List[Medium]:
    clouds = sweep_parameters(n_clouds, seed)
    meds = []
    for c in clouds:
        m = sweep_cloud_medium(c, tau_threshold)
        meds.append(m.with_packets(max(1, int(round(c.n_packets * packet_scale)))))
    return meds


def cube(n: int = 128, seed: int = 4, mean_tau_cell: float = 1.0e3, sigma_ln: float = 1.0,
         T: float = 1.0e4, sigma_v: float = 20.0, n_bins: int = 256, dv_bin: float = 25.0,
         tau_threshold: float = 10.0, n_sources: int = 64, packets_per_source: int = 1 << 18,
         name: str = "cube") -> Medium:
    """3D Cartesian cube of n^3 unit cells: ln k0 ~ N(ln mean - sigma^2/2, sigma) so that
    E[k0] = mean_tau_cell; Gaussian bulk velocity per component; bins uniform in velocity
    (dv_bin km/s); sources at the n_sources densest cells (ties to the lowest index)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ln_mu = math.log(mean_tau_cell) - 0.5 * sigma_ln * sigma_ln
    k0 = np.exp(rng.normal(ln_mu, sigma_ln, size=n * n * n))
    vel = rng.normal(0.0, sigma_v, size=(n * n * n, 3))
    dx = dv_bin / _vth_of_T(T)
    x_max = 0.5 * n_bins * dx
    order = np.argsort(-k0, kind="stable")[:n_sources]
    order = np.sort(order)
    iz, rem = np.divmod(order, n * n)
    iy, ix = np.divmod(rem, n)
    src = np.stack([ix + 0.5, iy + 0.5, iz + 0.5], axis=1).astype(np.float64)
    f = np.arange(n + 1, dtype=np.float64)
    return Medium(geometry=CART3D, n_cells=(n, n, n), faces=[f, f.copy(), f.copy()],
                  bin_edges=uniform_edges(x_max, n_bins), k0=k0,
                  temp=np.full(n * n * n, float(T)), vel=vel, src_pos=src,
                  src_x=np.zeros(len(src)), n_packets=int(n_sources * packets_per_source),
                  tau_threshold=float(tau_threshold), name=name)


def describe(m: Medium) -> dict:
    return {"name": m.name, "geometry": ["slab", "sphere", "cart3d"][m.geometry],
            "n_cells": list(m.n_cells), "n_bins": m.n_bins, "n_packets": m.n_packets,
            "tau0": float(np.max(m.k0)) if m.geometry != CART3D else None,
            "T": float(m.temp[0]), "tau_threshold": m.tau_threshold}
