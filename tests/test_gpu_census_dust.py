"""GPU time-dependent estimators (eq. 17: 'bin' counts at census times, 'path' residence
times per census interval), emission windows and dust (Sec. 2.4) against the exact chain's
transient law and absorption channel, the oracle walker, and exponential-integral transmission;
census tallies bit-identical across launch shapes and shard splits.

Bars: census counts are binomial (the 3 sigma rule per state and time); a residence-time
average lies in [0, 1] so its variance is at most its mean (5 such sigmas); fractions of
escaped and absorbed packets within 4 binomial sigmas."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import chain, walk1dh
from oracle import tables as tb
from paper_1709_10187_amd import media, rddmc
from tests._stats import assert_spectrum_matches, compare_exact, compare_two_samples

pytestmark = pytest.mark.gpu


def _gpu(m, n, seed=1):
    print(f"[census/dust] {m.name} cells={m.n_cells[0]} bins={m.n_bins} packets={n}", flush=True)
    p = rddmc.Problem(m.with_packets(n))
    p.run(seed=seed)
    return p.results()[0]


def _check_census(g, ex, n, edges):
    p = ex.at_edges.ravel()
    got = g.census_bin.ravel() / n
    assert np.all(got[p == 0] == 0)
    sig = np.sqrt(np.maximum(p * (1 - p), 1e-300) / n)
    z = np.abs(got - p) / np.where(p > 0, sig, 1.0)
    sel = p * n >= 10
    print(f"    census bin: {sel.sum()} cells, max |z| {z[sel].max():.2f}", flush=True)
    assert np.sum(z[sel] > 3) <= max(2, int(0.005 * sel.sum())) and z[sel].max() < 5
    dt = np.diff(edges)[:, None, None]
    mean = (g.census_path / rddmc.CENSUS_PATH_FIX / (n * dt)).ravel()
    want = ex.mean_in.ravel()
    tol = 5 * np.sqrt(np.maximum(want, 1e-30) / n) + 1e-6
    print(f"    census path: worst |err|/tol {np.max(np.abs(mean - want) / tol):.2f}", flush=True)
    assert np.all(np.abs(mean - want) <= tol)


@pytest.mark.parametrize("m", [media.slab(100.0, 1e4, 4, 6, x_max=4.0),
                               media.sphere(300.0, 1e4, 5, 8, x_max=5.0, v_max=12.0)], ids=["slab", "sphere_outflow"])
def test_census_estimators_match_exact_transient_law(m):
    ref = chain.solve(m)
    edges = np.array([0.0, 0.2, 0.5, 1.0, 2.0, 4.0]) * ref.t_mean
    n = 1 << 20
    g = _gpu(m.replace(census=edges), n)
    assert g.escaped == n
    _check_census(g, chain.transient(m, edges), n, edges)


def test_grey_diffusion_census_matches_the_continuous_time_walk():
    """The grey diffusion test (Sec. 3.1): 101 equal cells of a grey medium, a flash in the
    central cell, census at t = {1, 2, 4, 8, 16} x 1e-2 t_diff with t_diff = k R^2 / 2c; the
    bin and path estimators against the exact law of the discrete walk (the Bessel image sum
    of the grey chain, pinned in the oracle's tests)."""
    k = 1.0e3
    m = media.slab(k, 1e4, 101, 1, x_max=1.0)
    kbin = float(tb.build(m).k[0, 0])
    t_diff = kbin / 2.0
    edges = np.array([0.0, 1, 2, 4, 8, 16]) * 1e-2 * t_diff
    n = 1 << 20
    g = _gpu(m.replace(census=edges), n, seed=5)
    _check_census(g, chain.transient(m, edges), n, edges)


def test_emission_window_census_matches_exact_transient_law():
    m = media.slab(100.0, 1e4, 4, 6, x_max=4.0)
    ref = chain.solve(m)
    ts, te = 0.3 * ref.t_mean, 1.1 * ref.t_mean
    edges = np.array([0.0, 0.25, 0.5, 1.0, 1.5, 3.0]) * ref.t_mean
    n = 1 << 20
    g = _gpu(m.replace(census=edges, src_t=np.array([[ts, te]])), n, seed=7)
    _check_census(g, chain.transient(m, edges, emit=(ts, te)), n, edges)
    assert abs(g.t_mean - (ref.t_mean + 0.5 * (ts + te))) < 4.5 * math.sqrt(g.t_var / n)


def test_dust_in_ddmc_states_matches_exact_chain():
    m = media.sphere(400.0, 1e4, 6, 16, x_max=6.0, v_max=10.0)
    m = m.replace(dust_abs=np.linspace(0.5, 2.0, 6), dust_sca=np.full(6, 3.0))
    n = 1 << 20
    g = _gpu(m, n, seed=9)
    ref = chain.solve(m)
    assert g.escaped + g.absorbed == n and g.capped == 0
    pa = ref.absorbed
    print(f"    absorbed {g.absorbed / n:.5f} vs {pa:.5f}", flush=True)
    assert abs(g.absorbed / n - pa) < 4 * math.sqrt(pa * (1 - pa) / n)
    r = compare_exact(g.spectrum.ravel(), ref.spectrum.ravel() / ref.total, g.escaped)
    assert_spectrum_matches(r)
    assert abs(g.t_mean - ref.t_mean) < 4 * math.sqrt(ref.t_var / g.escaped)


@pytest.mark.parametrize("ka,ks", [(0.7, 0.0), (0.0, 0.7), (0.3, 0.4)])
def test_dust_in_mc_states_against_transmission(ka, ks):
    """Dust only (negligible Lya opacity, every state MC), central source in the slab |z| <= 1:
    one event with probability E_2(k) + (1 - E_2(k)) k_a / k, k = k_a + k_s."""
    m = media.slab(1e-9, 1e4, 1, 8, x_max=4.0, tau_threshold=1e30)
    m = m.replace(dust_abs=np.array([ka]), dust_sca=np.array([ks]))
    n = 1 << 21
    g = _gpu(m, n, seed=11)
    e2 = float(special.expn(2, ka + ks))
    p1 = e2 + (1.0 - e2) * ka / (ka + ks)
    assert abs(g.step_hist[0] / n - p1) <= 4 * math.sqrt(p1 * (1 - p1) / n)
    if ks == 0.0:
        assert abs(g.escaped / n - e2) < 4 * math.sqrt(e2 * (1 - e2) / n)
    if ka == 0.0:
        assert g.escaped == n
    assert g.escaped + g.absorbed == n
    spec = g.spectrum.sum(axis=0)
    assert spec[1 + 3] + spec[1 + 4] == g.escaped


def test_hybrid_dust_census_against_oracle_walker():
    """Everything at once on a moving hybrid slab (continuous-MC wings, dust, an emission window
    and a census): the GPU against the oracle walker as two samples (spectrum, absorbed
    fraction, census counts summed over bins)."""
    nc = 12
    m = media.slab(1e4, 1e4, nc, 48, x_max=16.0, tau_threshold=10.0, vel=np.linspace(-30, 30, nc))
    m = m.replace(dust_abs=np.full(nc, 0.8), dust_sca=np.full(nc, 2.0), src_t=np.array([[0.0, 2.0]]),
                  census=np.array([0.0, 1.0, 2.0, 4.0, 8.0]))
    ng, no = 1 << 18, 1 << 15
    g = _gpu(m, ng, seed=13)
    o = walk1dh.run(m, n_packets=no, seed=15)
    assert g.escaped + g.absorbed == ng and o.escaped + o.absorbed == no
    fa, fo = g.absorbed / ng, o.absorbed / no
    assert abs(fa - fo) < 4.5 * math.sqrt(fo * (1 - fo) * (1 / ng + 1 / no))
    assert_spectrum_matches(compare_two_samples(g.spectrum, o.spectrum))
    # census counts per (time, cell): two binomial samples
    gb = g.census_bin.sum(axis=2) / ng
    ob = o.e_bin.sum(axis=2) / no
    q = (gb * ng + ob * no) / (ng + no)
    sig = np.sqrt(np.maximum(q * (1 - q), 1e-300) * (1 / ng + 1 / no))
    z = np.abs(gb - ob) / np.where(q > 0, sig, 1.0)
    sel = q * no >= 10
    print(f"    census two-sample max |z| {z[sel].max():.2f} over {sel.sum()} cells", flush=True)
    assert z[sel].max() < 5 and np.sum(z[sel] > 3) <= 2


def _accel_batches(m, n, seeds):
    p = rddmc.Problem(m.with_packets(n))
    out = []
    for sd in seeds:
        p.reset()
        p.run(seed=sd)
        g = p.results()[0]
        assert g.escaped + g.absorbed + g.capped == n
        out.append(g.census_accel / rddmc.CENSUS_ACCEL_FIX / n)
    out = np.array(out)
    return out.mean(axis=0), out.std(axis=0, ddof=1) / math.sqrt(len(out))


@pytest.mark.parametrize("m", [media.sphere(400.0, 1e4, 4, 10, x_max=6.0, v_max=25.0),
                               media.slab(200.0, 1e4, 5, 8, x_max=5.0)], ids=["sphere_outflow", "slab"])
def test_acceleration_estimator_matches_exact_chain(m):
    """Eq. 18's optical-depth sums per cell and census interval (outward and inward leakage
    along the motion) against the chain's exact expectation: eight independent seeds of 2^17
    packets give the standard error; every cell within 5 of them."""
    ref = chain.solve(m)
    edges = np.array([0.0, 0.3, 1.0, 3.0, 10.0]) * ref.t_mean
    m = m.replace(census=edges)
    ex = chain.transient(m, edges).accel
    print(f"[census/dust] eq. 18 on {m.name}: 8 x 2^17 packets", flush=True)
    mean, se = _accel_batches(m, 1 << 17, range(21, 29))
    z = np.abs(mean - ex) / np.maximum(se, 1e-12)
    print(f"    max |z| {z.max():.2f}", flush=True)
    assert np.all(np.abs(mean - ex) <= 5.0 * se + 1e-7 * np.abs(ex).max())


def test_acceleration_grey_slab_net_crossings():
    """Steady eq. 18 on a grey slab whose every state has the same total rate K (vacuum faces
    leak at the interior rate): cell i collects (k/K)(2 P_top - 1{m > i} - 1{m >= i}) for a
    walk from cell m, P_top = m / (N + 1)."""
    N, start = 9, 3
    k = 50.0
    m0 = media.slab(k, 1e4, N, 1, x_max=1.0)
    dz = 2.0 / N
    t = tb.build(m0)
    kbin = float(t.k[0, 0])
    m = m0.replace(lam=kbin * dz / 2.0, src_pos=np.array([[-1 + dz * (start - 0.5), 0, 0]]))
    t = tb.build(m)
    K = float(t.K[0, 0])
    np.testing.assert_allclose(t.K[:, 0], K, rtol=1e-12)
    t_end = 400.0 * chain.solve(m).t_mean
    m = m.replace(census=np.array([0.0, t_end]))
    mean, se = _accel_batches(m, 1 << 17, range(31, 39))
    i = np.arange(1, N + 1)
    want = kbin / K * (2.0 * start / (N + 1.0) - (start > i) - (start >= i))
    print(f"    grey slab: max |z| {np.max(np.abs(mean[0] - want) / se[0]):.2f}", flush=True)
    assert np.all(np.abs(mean[0] - want) <= 5.0 * se[0] + 1e-6)


def test_census_tallies_bit_identical_across_launch_shapes_and_shards():
    """Census counts, residences and eq. 18 sums are integer sums, whatever a lane's path cache
    evicts when: launch shapes (block sizes give other lane-to-slot maps) and shard splits give
    the same bits."""
    m = media.slab(2e4, 1e4, 12, 48, x_max=20.0, tau_threshold=10.0).replace(
        census=np.array([0.0, 2.0, 5.0, 20.0, 80.0]), src_t=np.array([[0.0, 1.0]])).with_packets(1 << 13)
    print(f"[census/dust] bit identity: {m.name}, {m.n_packets} packets", flush=True)
    out = []
    for kw in (dict(), dict(block=64, grid=5, chunk=3), dict(block=192, grid=300, chunk=40)):
        p = rddmc.Problem(m)
        p.run(seed=13, **kw)
        out.append(p.tallies.cpu().numpy().copy())
    p = rddmc.Problem(m)
    for first, count in ((0, 3000), (3000, 7), (3007, 5185)):
        p.run(seed=13, first=first, count=count, block=128, chunk=17)
    out.append(p.tallies.cpu().numpy().copy())
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])
