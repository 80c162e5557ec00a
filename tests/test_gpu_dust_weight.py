"""GPU dust absorption by continuous packet weights (Sec. 2.4's second method): escaped weight
per slot against the killed chain's escape spectrum, the weighted mean escape time, the
weighted census and eq. 18 estimators with the path correction against the killed chain's
transient law (eq. 18 with leak probabilities r_f / K_leak: no absorption event ends a
weighted step), the hybrid walk (continuous-MC wings, frequency groups) against the oracle
walker's weight mode, and bit-identical tallies across launch shapes.

Bars: weighted spectra by the 3 sigma rule with each sample's own per-bin variance (from the
squared-weight spectrum); census and residence estimators within 5 sigma, their variance
bounded by their mean since weights lie in [0, 1]; eq. 18 within 5 standard errors of eight
seeds."""
import math

import numpy as np
import pytest

from oracle import chain, walk1dh
from paper_1709_10187_amd import media, rddmc
from tests._stats import assert_spectrum_matches, compare_weighted_exact, compare_weighted_two

pytestmark = pytest.mark.gpu

W = media.DUST_WEIGHT
BIN_FIX = float(1 << 24)   # weighted census counts: 2^-24 units


def _gpu(m, n, seed=1, **kw):
    print(f"[dust weights] {m.name} cells={m.n_cells[0]} bins={m.n_bins} packets={n} {kw}", flush=True)
    p = rddmc.Problem(m.with_packets(n))
    p.run(seed=seed, **kw)
    return p.results()[0]


def test_weighted_escapes_match_the_killed_chain():
    m = media.sphere(400.0, 1e4, 6, 16, x_max=6.0, v_max=10.0).replace(
        dust_abs=np.linspace(0.5, 2.0, 6), dust_sca=np.full(6, 3.0), flags=W)
    ref = chain.solve(m)
    n = 1 << 20
    g = _gpu(m, n, seed=3)
    assert g.escaped + g.absorbed == n and g.capped == 0 and g.absorbed < n // 100
    r = compare_weighted_exact(g.spectrum_w, g.spectrum_w2, n, ref.spectrum.ravel())
    esc = 1.0 - ref.absorbed
    sd = math.sqrt(max(g.spectrum_w2.sum() / n - (g.escaped_w / n) ** 2, 1e-300) / n)
    n_eff = g.escaped_w ** 2 / g.spectrum_w2.sum()
    print(f"    escaped weight {g.escaped_w / n:.5f} vs {esc:.5f}; max |z| {r['max_abs_z']:.2f} p {r['p_value']:.3g}; "
          f"t_w {g.t_mean_w:.5g} vs {ref.t_mean:.5g}", flush=True)
    assert_spectrum_matches(r)
    assert abs(g.escaped_w / n - esc) < 4 * sd
    assert abs(g.escaped_w - g.spectrum_w.sum()) < 1e-6 * n
    assert abs(g.t_mean_w - ref.t_mean) < 4.5 * math.sqrt(ref.t_var / n_eff)


def test_weighted_census_and_acceleration_match_the_killed_transient_law():
    m = media.slab(100.0, 1e4, 4, 6, x_max=4.0).replace(dust_abs=np.array([0.3, 0.8, 0.8, 0.3]),
                                                        dust_sca=np.full(4, 0.5), flags=W)
    ref = chain.solve(m)
    edges = np.array([0.0, 0.2, 0.5, 1.0, 2.0, 4.0]) * ref.t_mean
    ex = chain.transient(m, edges, dust_weights=True)
    m = m.replace(census=edges)
    n = 1 << 20
    g = _gpu(m, n, seed=5)
    p = ex.at_edges.ravel()
    got = g.census_bin.ravel() / BIN_FIX / n
    tol = 5 * np.sqrt(np.maximum(p, 1e-30) / n) + 1e-6
    print(f"    census bin: worst |err|/tol {np.max(np.abs(got - p) / tol):.2f}", flush=True)
    assert np.all(np.abs(got - p) <= tol)
    dt = np.diff(edges)[:, None, None]
    mean = (g.census_path / rddmc.CENSUS_PATH_FIX / (n * dt)).ravel()
    want = ex.mean_in.ravel()
    tol = 5 * np.sqrt(np.maximum(want, 1e-30) / n) + 1e-6
    print(f"    census path: worst |err|/tol {np.max(np.abs(mean - want) / tol):.2f}", flush=True)
    assert np.all(np.abs(mean - want) <= tol)
    prob = rddmc.Problem(m.with_packets(1 << 17))
    runs = []
    for sd in range(41, 49):
        prob.reset()
        prob.run(seed=sd)
        runs.append(prob.results()[0].census_accel / rddmc.CENSUS_ACCEL_FIX / (1 << 17))
    runs = np.array(runs)
    mean_a, se = runs.mean(axis=0), runs.std(axis=0, ddof=1) / math.sqrt(len(runs))
    print(f"    eq. 18: max |z| {np.max(np.abs(mean_a - ex.accel) / np.maximum(se, 1e-12)):.2f}", flush=True)
    assert np.all(np.abs(mean_a - ex.accel) <= 5.0 * se + 1e-7 * np.abs(ex.accel).max())


@pytest.mark.parametrize("name", ["hybrid_slab", "group_slab"])
def test_hybrid_weights_match_oracle_walker(name):
    base = media.slab(2e4, 1e4, 12, 48, x_max=20.0, tau_threshold=10.0)
    if name == "group_slab":
        base = media.slab(3e2, 1e4, 8, 24, x_max=12.0, tau_threshold=media.ALL_THIN, flags=media.GROUP_MC)
    m = base.replace(dust_abs=np.full(base.n_cells[0], 1.5), dust_sca=np.full(base.n_cells[0], 1.0),
                     flags=int(base.flags) | W)
    ng, no = 1 << 18, 1 << 14
    g = _gpu(m, ng, seed=7)
    o = walk1dh.run(m, n_packets=no, seed=29)
    r = compare_weighted_two(g.spectrum_w, g.spectrum_w2, ng, o.wspec, o.wspec2, no)
    print(f"    escaped weight {g.escaped_w / ng:.5f} vs {o.w_sum / no:.5f}; L1 {r['L1']:.4f} max |z| "
          f"{r['max_abs_z']:.2f} p {r['p_value']:.3g}; t_w {g.t_mean_w:.4g} vs {o.t_mean_w:.4g}", flush=True)
    assert_spectrum_matches(r)
    se = math.sqrt((g.spectrum_w2.sum() / ng - (g.escaped_w / ng) ** 2) / ng
                   + (o.wspec2.sum() / no - (o.w_sum / no) ** 2) / no)
    assert abs(g.escaped_w / ng - o.w_sum / no) < 4.5 * se


def test_weighted_tallies_are_bit_identical_across_launch_shapes():
    m = media.slab(2e4, 1e4, 12, 48, x_max=20.0, tau_threshold=10.0).replace(
        dust_abs=np.full(12, 1.5), dust_sca=np.full(12, 1.0), flags=W, census=np.array([0.0, 5.0, 20.0, 80.0]))
    out = []
    for kw in (dict(), dict(block=64, grid=5, chunk=3), dict(block=256, grid=300, chunk=40)):
        p = rddmc.Problem(m.with_packets(1 << 13))
        p.run(seed=9, **kw)
        out.append(p.tallies.cpu().numpy().copy())
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])
