"""Pins of the 1D hybrid oracle walker (O1-1DH, slabs and spherical shells): pure mode against
the exact chain, slabs against the independently written 3D walker on slab-shaped boxes
(all-MC, hybrid, moving, non-uniform), the shell geometry against free-streaming quadratures,
all-MC spheres against the derived sphere spectrum, the core-skipping draw against its
moment identity, the census estimators and emission windows against the exact transient law,
and dust against the chain's absorption channel and exponential-integral transmission."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import analytic as an
from oracle import chain, linemath, walk1dh, walk3d
from paper_1709_10187_amd import media
from tests._stats import assert_spectrum_matches, compare_exact, compare_two_samples


@pytest.mark.parametrize("m", [media.slab(300.0, 1e4, 8, 16, x_max=6.0),
                               media.sphere(1e3, 1e4, 8, 24, x_max=8.0, v_max=20.0)], ids=["slab", "sphere_outflow"])
def test_pure_mode_matches_exact_chain(m):
    n = 100000
    r = walk1dh.run(m, n_packets=n, seed=1)
    ref = chain.solve(m)
    assert r.escaped == n and r.to_mc == 0
    assert_spectrum_matches(compare_exact(r.spectrum, ref.spectrum, n))
    assert abs(r.steps_mean - ref.steps) < 4 * math.sqrt(ref.steps_var / n)
    assert abs(r.t_mean - ref.t_mean) < 4 * math.sqrt(ref.t_var / n)


def _slab_box(m1, width=1.0e6):
    """The same slab as a 3D grid of 1 x 1 x n cells of lateral extent 2 width."""
    nz = m1.n_cells[0]
    fx = np.array([-width, width])
    vel = None if m1.vel is None else np.stack([np.zeros(nz), np.zeros(nz), np.asarray(m1.vel)], axis=1)
    return media.Medium(geometry=2, n_cells=(1, 1, nz), faces=[fx, fx.copy(), np.asarray(m1.faces[0])],
                        bin_edges=m1.bin_edges, k0=m1.k0, temp=m1.temp, vel=vel,
                        src_pos=np.array([[0.0, 0.0, float(m1.src_pos[0][0])]]), src_x=m1.src_x,
                        n_packets=m1.n_packets, tau_threshold=m1.tau_threshold, lam=m1.lam, name="slab_box")


SLABS = {
    "all_mc": media.slab(4e2, 1e4, 16, 64, x_max=20.0, tau_threshold=1e30),
    "hybrid": media.slab(2e4, 1e4, 16, 64, x_max=20.0, tau_threshold=10.0),
    "hybrid_moving": media.slab(2e4, 1e4, 16, 64, x_max=20.0, tau_threshold=10.0, vel=np.linspace(-40, 40, 16)),
    "hybrid_nonuniform_hot_cold": media.slab(2e4, 1e4, 16, 64, x_max=20.0, tau_threshold=5.0).replace(
        k0=2e4 * np.exp(np.sin(np.arange(16) * 1.3)), temp=1e4 * np.exp(0.5 * np.cos(np.arange(16) * 0.7))),
}


@pytest.mark.parametrize("name", sorted(SLABS))
def test_slab_matches_3d_walker_on_a_slab_box(name):
    """Two independently written geometries of the same slab: the 1D walker's planes against the
    3D walker's Cartesian box (its lateral walls 1e6 away); escape spectra as two samples,
    escape times and conversion counts within their noise."""
    m1 = SLABS[name]
    n = 20000
    a = walk1dh.run(m1, n_packets=n, seed=3)
    b = walk3d.run(_slab_box(m1), n_packets=n, seed=4)
    assert a.escaped == n and b.escaped == n
    assert b.spectrum[:4].sum() <= 2
    assert_spectrum_matches(compare_two_samples(a.spectrum.sum(axis=0), b.spectrum[4:6].sum(axis=0)))
    # face split: both rows
    fa, fb = a.spectrum.sum(axis=1), b.spectrum[4:6].sum(axis=1)
    assert abs(fa[0] / n - fb[0] / n) < 4 * math.sqrt(0.5 / n)
    se = math.sqrt((a.t_var + b.t_var) / n)
    assert abs(a.t_mean - b.t_mean) < 4 * se
    for x, y in ((a.to_mc, b.to_mc), (a.to_ddmc, b.to_ddmc), (a.reflected, b.reflected)):
        # counts per packet are heavy-tailed: compare within 6 Poisson-like sigmas plus 2 %
        assert abs(x - y) <= 6 * math.sqrt(x + y + 1) + 0.02 * (x + y), (x, y)


def _free_streaming_mean(r0):
    """Mean distance from a point at radius r0 to the unit sphere along an isotropic ray."""
    f = lambda mu: -r0 * mu + math.sqrt(r0 * r0 * mu * mu - r0 * r0 + 1.0)
    return 0.5 * integrate.quad(f, -1.0, 1.0, epsabs=0, epsrel=1e-12)[0]


@pytest.mark.parametrize("r0", [0.0, 0.37, 0.8])
def test_shell_geometry_free_streaming(r0):
    """An optically thin sphere of 40 shells (all states MC): unscattered packets cross many shell
    boundaries; the mean escape time is the mean chord from the source to r = 1, and the face
    crossing leaves the comoving frequency of a static sphere unchanged."""
    m = media.sphere(1e-7, 1e4, 40, 16, x_max=4.0, tau_threshold=1e30).replace(src_pos=np.array([[r0, 0.0, 0.0]]))
    n = 200000
    r = walk1dh.run(m, n_packets=n, seed=9)
    assert r.escaped == n
    assert r.steps_mean >= 40 * (1 - r0) - 1e-9            # at least one event per shell crossed outward
    want = _free_streaming_mean(r0)
    sd = math.sqrt(max(r.t_var, 1e-30) / n)
    assert abs(r.t_mean - want) < max(4 * sd, 1e-9), (r.t_mean, want)
    spec = r.spectrum.sum(axis=0)
    assert spec[1 + 8] + spec[1 + 7] == n                  # x = 0 stays at the centre bins


def test_all_mc_sphere_matches_derived_spectrum():
    """Brute-force MCRT in a uniform sphere at a tau0 = 1e3 (T = 0.1 K, a = 0.149): the escape
    spectrum against the derived sphere solution, with the exact chain's own distance to it at
    the same a tau0 (200 shells x 240 bins folded onto the tally grid) plus twice the noise as
    the bar."""
    atau0, T, nb = 1.0e3, 0.1, 48
    a = float(linemath.damping(np.array([T]))[0])
    tau0 = atau0 / a
    s = atau0 ** (1.0 / 3.0)
    n = 1 << 13
    m = media.sphere(tau0, T, 1, nb, x_max=4.0 * s, tau_threshold=1e30, n_packets=n)
    r = walk1dh.run(m, n_packets=n, seed=2)
    assert r.escaped == n and r.to_ddmc == 0
    cnt = r.spectrum.sum(axis=0)
    assert cnt[0] == 0 and cnt[-1] == 0
    p = cnt[1:-1] / n
    ref = an.binned(an.sphere_pdf, m.bin_edges, atau0)
    mo = media.sphere(tau0, T, 200, nb * 5, x_max=4.0 * s)
    po = chain.solve(mo).spectrum_total()[1:-1].reshape(nb, 5).sum(axis=1)
    noise = float(np.sum(np.sqrt(2.0 / np.pi * po * (1.0 - po) / n)))
    l1_mc, l1_chain = float(np.abs(p - ref).sum()), float(np.abs(po - ref).sum())
    assert l1_mc <= l1_chain + 2.0 * noise, (l1_mc, l1_chain, noise)
    half = compare_two_samples(cnt[1:-1][:nb // 2], cnt[1:-1][nb // 2:][::-1])
    assert_spectrum_matches(half)


@pytest.mark.parametrize("x_crit", [0.0, 3.0])
def test_core_skipping_moment_identity(x_crit):
    """Second moment of the frequency change of a core scattering (|x| < x_crit):
    E[(x' - x)^2] = (4/3) E[u_par^2] + (1/3) (x_crit^2 + 1): the parallel term with
    E[(mu - 1)^2] = 4/3, the perpendicular one with E[1 - mu^2] = 2/3 and E[u_perp^2] =
    (x_crit^2 + 1)/2 for the projection of a 2D speed whose square exceeds x_crit^2 by an
    Exp(1) variable (a 2D Maxwellian without its core)."""
    a, x = 4.702e-4, 1.2
    n = 400000
    d = walk3d.redistribution_samples(a, x, n, seed=17, x_crit=x_crit) - x
    f = lambda u: math.exp(-u * u) / (a * a + (x - u) ** 2)
    Z = integrate.quad(f, -12, 12, points=[x], limit=400)[0]
    eu2 = integrate.quad(lambda u: u * u * f(u), -12, 12, points=[x], limit=400)[0] / Z
    want = 4.0 / 3.0 * eu2 + (x_crit * x_crit + 1.0) / 3.0
    se = (d ** 2).std() / math.sqrt(n)
    assert abs((d ** 2).mean() - want) < 4 * se, ((d ** 2).mean(), want, se)


def _census_checks(m, edges, n, emit=None):
    """The walker's census counts and residence times against the exact transient law: the bin
    estimator is a binomial count; the path estimator averages a variable in [0, 1] whose
    variance is at most its mean."""
    r = walk1dh.run(m.replace(census=edges), n_packets=n, seed=13)
    ex = chain.transient(m, edges, emit=emit)
    p = ex.at_edges.ravel()
    got = r.e_bin.ravel() / n
    sig = np.sqrt(np.maximum(p * (1 - p), 1e-300) / n)
    z = np.abs(got - p) / np.where(p > 0, sig, 1.0)
    assert np.all(got[p == 0] == 0)
    assert np.sum(z[p * n >= 10] > 3) <= 2 and z[p * n >= 10].max() < 5, z.max()
    dt = np.diff(edges)[:, None, None]
    mean = (r.e_path / (n * dt)).ravel()
    want = ex.mean_in.ravel()
    assert np.all(np.abs(mean - want) <= 5 * np.sqrt(np.maximum(want, 1e-30) / n) + 1e-12)
    return r, ex


@pytest.mark.parametrize("m", [media.slab(100.0, 1e4, 4, 6, x_max=4.0),
                               media.sphere(300.0, 1e4, 5, 8, x_max=5.0, v_max=12.0)], ids=["slab", "sphere_outflow"])
def test_census_estimators_match_exact_transient_law(m):
    ref = chain.solve(m)
    edges = np.array([0.0, 0.2, 0.5, 1.0, 2.0, 4.0]) * ref.t_mean
    _census_checks(m, edges, 200000)


def test_emission_window_census_matches_exact_transient_law():
    m = media.slab(100.0, 1e4, 4, 6, x_max=4.0)
    ref = chain.solve(m)
    ts, te = 0.3 * ref.t_mean, 1.1 * ref.t_mean
    edges = np.array([0.0, 0.25, 0.5, 1.0, 1.5, 3.0]) * ref.t_mean
    r, _ = _census_checks(m.replace(src_t=np.array([[ts, te]])), edges, 200000, emit=(ts, te))
    # escape times are emission time plus the flash law's: their mean shifts by (ts + te) / 2
    se = math.sqrt(r.t_var / r.escaped)
    assert abs(r.t_mean - (ref.t_mean + 0.5 * (ts + te))) < 4.5 * se


def test_dust_in_ddmc_states_matches_exact_chain():
    """Dust absorption as a competing exponential in every DDMC step, with dust scattering in
    the leakage coefficients: escape and absorption fractions and the spectrum of the escaped
    packets against the chain's absorption channel."""
    m = media.sphere(400.0, 1e4, 6, 16, x_max=6.0, v_max=10.0)
    m = m.replace(dust_abs=np.linspace(0.5, 2.0, 6), dust_sca=np.full(6, 3.0))
    n = 200000
    r = walk1dh.run(m, n_packets=n, seed=21)
    ref = chain.solve(m)
    assert r.escaped + r.absorbed == n
    pa = ref.absorbed
    assert abs(r.absorbed / n - pa) < 4 * math.sqrt(pa * (1 - pa) / n)
    assert_spectrum_matches(compare_exact(r.spectrum.ravel(), ref.spectrum.ravel() / ref.total, r.escaped))
    assert abs(r.t_mean - ref.t_mean) < 4 * math.sqrt(ref.t_var / r.escaped)


@pytest.mark.parametrize("ka,ks", [(0.7, 0.0), (0.0, 0.7), (0.3, 0.4)])
def test_dust_in_mc_states_against_transmission(ka, ks):
    """A slab |z| <= 1 of dust only (negligible Lya opacity, every state MC), source at the
    centre: a packet leaves with no interaction with probability E_2(k_a + k_s) (the
    exponential integral: isotropic directions through an optical depth k / |mu|), and its
    first interaction is an absorption with probability k_a / (k_a + k_s), so it takes one
    event with probability E_2 + (1 - E_2) k_a / (k_a + k_s); with no scattering E_2 is the
    escape fraction, with no absorption every packet escapes."""
    m = media.slab(1e-9, 1e4, 1, 8, x_max=4.0, tau_threshold=1e30)
    m = m.replace(dust_abs=np.array([ka]), dust_sca=np.array([ks]))
    n = 400000
    r = walk1dh.run(m, n_packets=n, seed=3)
    e2 = float(special.expn(2, ka + ks))
    p1 = e2 + (1.0 - e2) * ka / (ka + ks)
    one_step = r.step_hist[0] / n
    assert abs(one_step - p1) <= 4 * math.sqrt(p1 * (1 - p1) / n)
    if ks == 0.0:
        assert abs(r.escaped / n - e2) < 4 * math.sqrt(e2 * (1 - e2) / n)
    if ka == 0.0:
        assert r.escaped == n
    assert r.escaped + r.absorbed == n
    spec = r.spectrum.sum(axis=0)
    assert spec[1 + 3] + spec[1 + 4] == r.escaped              # dust scattering keeps x = 0
