"""Pins of the 3D hybrid oracle walker (O1-3D): its own Dawson/Voigt, the atom-velocity
sampler, the interface conversion probability, continuous-MC geometry and opacity against
independent quadratures, the whole scattering against the textbook redistribution function,
brute-force MCRT of the slab against eq. 33, and pure-DDMC runs against the exact chain."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import analytic as an
from oracle import chain, linemath, walk3d
from paper_1709_10187_amd import media
from tests._stats import assert_spectrum_matches, compare_exact, compare_two_samples


def test_own_dawson_and_voigt():
    xs = np.concatenate([np.linspace(-30, 30, 301), [1e-4, 0.2, 5.999, 6.0, 6.001, 80.0, 1e4]])
    for x in xs:
        if x == 0:
            continue
        assert walk3d.dawson(x) == pytest.approx(special.dawsn(x), rel=1e-13)
        assert walk3d.voigt(4.702e-4, x) == pytest.approx(float(linemath.voigt_H(4.702e-4, x)), rel=1e-11,
                                                          abs=1e-300)


@pytest.mark.parametrize("a,x", [(4.702e-4, 0.0), (4.702e-4, 1.7), (4.702e-4, 3.0), (4.702e-4, -6.0),
                                 (1.4869e-2, 2.2), (4.702e-4, 25.0)])
def test_atom_velocity_sampler_matches_density(a, x):
    """u_par ~ exp(-u^2) / (a^2 + (x - u)^2) (the parallel atom velocity of a scattering at
    frequency x; the paper's density without its missing minus sign)."""
    n = 200000
    smp = walk3d.upar_samples(a, x, n, seed=11)
    f = lambda u: math.exp(-u * u) / (a * a + (x - u) ** 2)
    lo, hi = np.percentile(smp, [0.5, 99.5])
    edges = np.linspace(lo, hi, 31)
    cnt, _ = np.histogram(smp, edges)
    Z = integrate.quad(f, -20, 20 + abs(x), points=[x], limit=800)[0]
    p = np.array([integrate.quad(f, edges[i], edges[i + 1], limit=200,
                                 points=[x] if edges[i] < x < edges[i + 1] else None)[0] for i in range(30)]) / Z
    z = (cnt / n - p) / np.sqrt(p * (1 - p) / n)
    assert np.sum(np.abs(z) > 3) <= 2 and np.abs(z).max() < 5


def test_interface_conversion_probability_needs_tau_at_least_two():
    """P = 2/(tau + 2 lambda) (2/3 + mu) <= 1 for every mu in (0, 1] iff tau >= 10/3 - 2 lambda
    (~1.91), the hybrid section's 'tau_DDMC >~ 2' condition."""
    lam = 0.7104
    P = lambda tau, mu: 2.0 / (tau + 2 * lam) * (2.0 / 3.0 + mu)
    assert P(2.0, 1.0) <= 1.0 and P(1.85, 1.0) > 1.0
    assert abs((10.0 / 3.0 - 2 * lam) - 1.9125) < 1e-3


def _uniform_cube(n, tau_cell, nb=8, dv=25.0, tau_th=1e30, packets=20000):
    m = media.cube(n=n, seed=1, mean_tau_cell=tau_cell, sigma_ln=1e-9, sigma_v=0.0, n_bins=nb + 1, dv_bin=dv,
                   tau_threshold=tau_th, n_sources=1, packets_per_source=packets)
    c = n // 2
    return m.replace(k0=np.full(n ** 3, float(tau_cell)), vel=None, src_pos=np.array([[c + 0.5] * 3]))


def test_free_streaming_escape_time():
    """Optically thin cube, all-MC (tau_th huge): packets fly straight from the centre; the mean
    escape time is (L/2) E[1 / max_i |n_i|] over isotropic n (independent quadrature)."""
    n = 5
    m = _uniform_cube(n, 1e-7, packets=40000)
    r = walk3d.run(m, seed=3)
    assert r.escaped == 40000 and r.reflected == 0
    f = lambda th, ph: 1.0 / max(abs(math.sin(th) * math.cos(ph)), abs(math.sin(th) * math.sin(ph)),
                                 abs(math.cos(th))) * math.sin(th) / (4 * math.pi)
    E, _ = integrate.dblquad(lambda th, ph: f(th, ph), 0, 2 * math.pi, 0, math.pi, epsabs=1e-7)
    ref = 0.5 * n * E
    assert r.t_mean == pytest.approx(ref, rel=4 * (0.3 / math.sqrt(40000)) + 1e-3)
    # no scattering: the escape spectrum is the source line, all in the central bin
    assert r.spectrum.sum(axis=0)[1 + 4] == 40000


def test_unscattered_escape_fraction():
    """P(no scattering before escape) = E[exp(-k0 H(a,0) d(n))] from the centre of a uniform
    cube: checks the MC opacity k0 H(a,x) and the exponential path sampling."""
    n = 1                      # one cell: the first event is a scattering or the escape
    tau = 0.4
    m = _uniform_cube(n, tau, packets=100000)
    r = walk3d.run(m, seed=5, max_steps=1)
    k = tau * float(linemath.voigt_H(float(linemath.damping(1e4)), 0.0))

    def d(th, ph):
        nn = (abs(math.sin(th) * math.cos(ph)), abs(math.sin(th) * math.sin(ph)), abs(math.cos(th)))
        return 0.5 * n / max(nn)

    P, _ = integrate.dblquad(lambda th, ph: math.exp(-k * d(th, ph)) * math.sin(th) / (4 * math.pi),
                             0, 2 * math.pi, 0, math.pi, epsabs=1e-8)
    frac = r.escaped / 100000
    assert abs(frac - P) < 4 * math.sqrt(P * (1 - P) / 100000)


def test_pure_ddmc_cube_matches_exact_chain():
    m = media.cube(n=5, seed=7, mean_tau_cell=300.0, n_bins=16, dv_bin=25.0, tau_threshold=0.0, n_sources=2,
                   packets_per_source=30000)
    r = walk3d.run(m, seed=1)
    c = chain.solve(m)
    res = compare_exact(r.spectrum, c.spectrum, r.n_packets)
    assert_spectrum_matches(res)
    assert abs(r.steps_mean - c.steps) < 4 * math.sqrt(c.steps_var / r.n_packets)
    assert abs(r.t_mean - c.t_mean) < 4 * math.sqrt(c.t_var / r.n_packets)
    assert r.to_mc == 0 and r.pixels.sum() == r.n_packets


def test_lab_escape_law_quadrature_against_sampling():
    rng = np.random.default_rng(1)
    n = 1_000_000
    e = np.linspace(-5, 5, 21)
    lo, hi, un, ut = 0.0, 0.5, 0.7, 1.3
    x = rng.uniform(lo, hi, n)
    mu = rng.uniform(0, 1, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    xl = x + mu * un + np.sqrt(1 - mu * mu) * ut * np.cos(ph)
    cnt = np.bincount(np.clip(np.searchsorted(e, xl, side="right"), 0, 21), minlength=22) / n
    p = chain.lab_bin_probs_3d(e, lo, hi, un, ut)
    assert p.sum() == pytest.approx(1.0, abs=1e-12)
    assert np.all(p >= 0.0)
    assert np.all(np.abs(cnt - p) < 5 * np.sqrt(p * (1 - p) / n) + 1e-6)


def _hummer_r2a(a, x, xp):
    """Hummer's (1962) angle-averaged redistribution function for natural plus Doppler
    broadening and an isotropic phase function (R_II-A): the joint density of absorption at
    x and re-emission at x' in the observer's frame; its integral over x' is H(a,x)/sqrt(pi)."""
    lo, hi = min(x, xp), max(x, xp)
    f = lambda u: math.exp(-u * u) * (math.atan((lo + u) / a) - math.atan((hi - u) / a))
    v, _ = integrate.quad(f, 0.5 * (hi - lo), np.inf, limit=400, epsabs=0, epsrel=1e-10)
    return v / math.pi ** 1.5


@pytest.mark.parametrize("a,x", [(1.4869e-2, 0.5), (1.4869e-2, 3.0), (4.702e-4, 8.0), (0.1487, 5.0)])
def test_scattering_redistribution_matches_hummer_r2a(a, x):
    """The walker's whole scattering (atom velocity along the photon from its rejection
    sampler, one perpendicular component from N(0, 1/2), an isotropic new direction and the
    eq. 41 frequency with no recoil) against the textbook redistribution law:
    p(x' | x) = sqrt(pi) R_II-A(x, x') / H(a, x), with H the exact Voigt function.  A dropped
    perpendicular term, a wrong sign of u_par or of (mu - 1), or an anisotropic direction
    each change this law."""
    n = 200000
    smp = walk3d.redistribution_samples(a, x, n, seed=5)
    lo, hi = np.percentile(smp, [0.5, 99.5])
    edges = np.linspace(lo, hi, 31)
    cnt, _ = np.histogram(smp, edges)
    H = special.wofz(x + 1j * a).real
    g = lambda xp: _hummer_r2a(a, x, xp)
    p = np.array([integrate.quad(g, edges[i], edges[i + 1], limit=100,
                                 points=[x] if edges[i] < x < edges[i + 1] else None)[0]
                  for i in range(30)]) * math.sqrt(math.pi) / H
    assert 0.0 < 1.0 - p.sum() < 0.02          # the law is normalised; ~1 % lies outside
    res = compare_exact(np.r_[cnt, n - cnt.sum()], np.r_[p, 1.0 - p.sum()])
    assert_spectrum_matches(res)


def _all_mc_slab(atau0, T, n_bins, x_max, packets, width=1.0e3):
    """The slab |z| <= 1 as one 3D cell of lateral extent 2 width (packets leave through the
    z faces), with every state a continuous-MC state (tau_th above every state's depth): the
    walker is then brute-force Monte Carlo transfer, scattering by scattering."""
    a = float(linemath.damping(np.array([T]))[0])
    tau0 = atau0 / a
    fz = np.array([-1.0, 1.0])
    fx = np.array([-width, width])
    m = media.Medium(geometry=2, n_cells=(1, 1, 1), faces=[fx, fx.copy(), fz],
                     bin_edges=media.uniform_edges(x_max, n_bins), k0=np.array([tau0]), temp=np.array([T]),
                     vel=None, src_pos=np.array([[0.0, 0.0, 0.0]]), src_x=np.array([0.0]), n_packets=packets,
                     tau_threshold=1.0e30, name="all_mc_slab")
    return m, tau0


def test_all_mc_slab_escape_spectrum_matches_neufeld():
    """Brute-force MCRT of the Neufeld problem (Sec. 3.2.1, eq. 33) at a tau0 = 1e3 (T = 0.1 K,
    a = 0.149, tau0 = 6725: ~1.2e4 scatterings per packet).  Eq. 33 is the large-a tau0 limit,
    so at this depth the exact solution differs from it; the bar is the exact chain's own
    distance to eq. 33 at the same a tau0 (201 cells x 240 bins, folded onto the tally grid)
    plus twice the expected Monte Carlo noise L1.  Exact properties of the static problem are
    checked as well: both faces equally likely, the spectrum symmetric in x."""
    atau0, T, nb = 1.0e3, 0.1, 48
    s = atau0 ** (1.0 / 3.0)
    n = 1 << 14
    m, tau0 = _all_mc_slab(atau0, T, nb, 4.0 * s, n)
    r = walk3d.run(m, n_packets=n, seed=1)
    assert r.escaped == n and r.to_ddmc == 0 and r.to_mc == 0
    faces = r.spectrum.sum(axis=1)
    assert faces[:4].sum() == 0
    assert abs(faces[4] - faces[5]) < 4.0 * math.sqrt(n)            # Binomial(n, 1/2)
    cnt = r.spectrum.sum(axis=0)
    assert cnt[0] == 0 and cnt[-1] == 0
    cnt = cnt[1:-1]
    p = cnt / n
    ref = an.binned(an.slab_pdf, m.bin_edges, atau0)
    mo = media.slab(tau0, T, 201, nb * 5, x_max=4.0 * s)
    po = chain.solve(mo).spectrum_total()[1:-1].reshape(nb, 5).sum(axis=1)
    noise = float(np.sum(np.sqrt(2.0 / np.pi * po * (1.0 - po) / n)))
    l1_mc, l1_chain = float(np.abs(p - ref).sum()), float(np.abs(po - ref).sum())
    assert l1_mc <= l1_chain + 2.0 * noise, (l1_mc, l1_chain, noise)
    # mirror symmetry x -> -x: the two halves are two samples of the same law
    half = compare_two_samples(cnt[:nb // 2], cnt[nb // 2:][::-1])
    assert_spectrum_matches(half)
