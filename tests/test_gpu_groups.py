"""GPU frequency-group Monte Carlo (Sec. 5.3): the discrete redistribution tables of eq. 42
against O6 (element by element, FP64 quadrature against QUADPACK), their mirror symmetry and
row sums, the alias tables against the rows they encode, and the walk against the 1D oracle
walker's group mode (escape spectra as two samples by the 3 sigma rule, mean escape times and
event counts within their noise) and against the single-scattering limit (E_2 and O6's row).

Bars: table elements within 1e-7 relative (plus 1e-18 absolute) of O6 at epsrel 1e-9 (the
kernel's rule is converged to ~1e-9, measured against O6 at 1e-10); rows sum to 1 within 1e-8;
mirror pairs agree within 1e-9 relative; the alias tables reproduce their normalised rows within
nb 2^-32 per entry."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import redistribution as rd
from oracle import tables as tb
from oracle import walk1dh
from paper_1709_10187_amd import media, rddmc
from tests._stats import assert_spectrum_matches, compare_two_samples

pytestmark = pytest.mark.gpu

G = media.GROUP_MC
THIN = media.ALL_THIN
CASES = {
    "slab_groups": media.slab(3e2, 1e4, 8, 24, x_max=12.0, tau_threshold=THIN, flags=G),
    "sphere_groups": media.sphere(3e2, 1e4, 8, 24, x_max=12.0, tau_threshold=THIN, flags=G),
    "slab_hybrid_groups": media.slab(2e4, 1e4, 16, 41, x_max=20.0, tau_threshold=10.0, flags=G),
    "sphere_hybrid_groups_cold": media.sphere(1e4, 1e2, 12, 61, x_max=30.0, tau_threshold=10.0, flags=G),
    "slab_groups_dust": media.slab(3e2, 1e4, 8, 24, x_max=12.0, tau_threshold=THIN, flags=G).replace(
        dust_abs=np.full(8, 0.2), dust_sca=np.full(8, 0.3)),
}


def test_tables_match_the_oracle():
    m = CASES["slab_groups"]
    p = rddmc.Problem(m)
    prob, alias = p.read_redistribution(0)
    nb = m.n_bins
    a = media._a_of_T(1e4)
    print(f"[groups] {nb} bins, a = {a:.4g}: row sums {prob.sum(axis=1).min():.12f} .. {prob.sum(axis=1).max():.12f}",
          flush=True)
    worst = 0.0
    for jp, j in [(12, 12), (12, 11), (11, 13), (0, 0), (0, 1), (23, 20), (5, 5), (5, 9), (17, 2)]:
        want = rd.group_probability(m.bin_edges, a, jp, j, epsrel=1e-9)
        err = abs(prob[jp, j] - want)
        if want > 1e-18:
            worst = max(worst, err / want)
        assert err <= 1e-7 * want + 1e-18, (jp, j, prob[jp, j], want)
    print(f"    worst relative difference to O6 over the sampled elements {worst:.2e}", flush=True)
    np.testing.assert_allclose(prob.sum(axis=1), 1.0, atol=1e-8)
    mirror = prob[::-1, ::-1]
    np.testing.assert_allclose(prob, mirror, rtol=1e-9, atol=1e-20)
    # the alias tables encode the normalised rows
    q = prob / prob.sum(axis=1, keepdims=True)
    thr = alias[..., 0].astype(np.float64) / 2.0 ** 32
    rec = np.zeros_like(q)
    rows = np.arange(nb)[:, None]
    np.add.at(rec, (np.broadcast_to(rows, (nb, nb)), np.broadcast_to(np.arange(nb), (nb, nb))), thr / nb)
    np.add.at(rec, (np.broadcast_to(rows, (nb, nb)), alias[..., 1].astype(np.int64)), (1.0 - thr) / nb)
    assert np.all(alias[..., 1] < nb)
    np.testing.assert_allclose(rec, q, rtol=0, atol=nb * 2.0 ** -32)


def test_tables_of_an_efficient_grid():
    """Odd bin count, a wide central bin and unit wings (the paper's efficient grid): rows sum
    to 1 and the central bin's self-transition matches O6."""
    a = media._a_of_T(1e4)
    edges = media.efficient_edges(a, 1e5, 1.0 / 64)
    m = media.slab(1e5, 1e4, 64, len(edges) - 1, tau_threshold=THIN, flags=G).replace(bin_edges=edges)
    prob, _ = rddmc.Problem(m).read_redistribution(0)
    c = (len(edges) - 1) // 2
    np.testing.assert_allclose(prob.sum(axis=1), 1.0, atol=1e-8)
    for jp, j in [(c, c), (c, c + 1), (c + 3, c + 2)]:
        want = rd.group_probability(edges, a, jp, j, epsrel=1e-9)
        assert abs(prob[jp, j] - want) <= 1e-7 * want + 1e-18, (jp, j, prob[jp, j], want)


def test_tables_of_a_cold_fine_grid():
    """T = 100 K (a = 4.7e-3) on 201 bins of width 0.2 over |x| <= 20, finer than the unit
    width of wing redistribution: rows sum to 1, the mirror symmetry holds, and core, wing and
    edge elements match O6."""
    a = media._a_of_T(1e2)
    m = media.slab(3e2, 1e2, 8, 201, x_max=20.0, tau_threshold=THIN, flags=G)
    prob, _ = rddmc.Problem(m).read_redistribution(0)
    np.testing.assert_allclose(prob.sum(axis=1), 1.0, atol=1e-8)
    np.testing.assert_allclose(prob, prob[::-1, ::-1], rtol=1e-9, atol=1e-20)
    for jp, j in [(100, 100), (100, 101), (100, 96), (180, 178), (0, 0)]:
        want = rd.group_probability(m.bin_edges, a, jp, j, epsrel=1e-9)
        assert abs(prob[jp, j] - want) <= 1e-7 * want + 1e-18, (jp, j, prob[jp, j], want)


def test_table_build_of_a_wide_grid():
    """1024 bins of width 0.078 over |x| <= 40 (the widest grids of the batched sweep): rows sum
    to 1; the build time is printed (pairs of bins more than 13 apart are skipped)."""
    import time
    import torch
    m = media.slab(3e2, 1e4, 4, 1024, x_max=40.0, tau_threshold=THIN, flags=G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = rddmc.Problem(m)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prob, _ = p.read_redistribution(0)
    print(f"[groups] 1024-bin tables built in {dt:.2f} s", flush=True)
    np.testing.assert_allclose(prob.sum(axis=1), 1.0, atol=1e-8)


def test_unsupported_clouds_are_refused():
    for bad in (CASES["slab_groups"].replace(vel=np.linspace(-5, 5, 8)),
                CASES["slab_groups"].replace(temp=np.linspace(1e4, 2e4, 8)),
                CASES["slab_groups"].replace(tau_threshold=0.0)):
        with pytest.raises(RuntimeError):
            rddmc.Problem(bad)


@pytest.mark.parametrize("name", sorted(CASES))
def test_group_walk_matches_oracle_walker(name):
    m = CASES[name]
    ng, no = 1 << 18, 1 << 14
    print(f"[groups] {name}: cells={m.n_cells[0]} bins={m.n_bins} tau_th={m.tau_threshold:.3g} packets {ng} / {no}",
          flush=True)
    p = rddmc.Problem(m.with_packets(ng))
    p.run(seed=2)
    g = p.results()[0]
    o = walk1dh.run(m, n_packets=no, seed=9)
    ng_out = g.escaped + g.absorbed
    assert g.launched == ng and ng_out == ng and g.capped == 0
    assert o.escaped + o.absorbed == no
    r = compare_two_samples(g.spectrum, o.spectrum)
    print(f"    L1 {r['L1']:.4f} max|z| {r['max_abs_z']:.2f} p {r['p_value']:.3g}; t {g.t_mean:.4g} vs {o.t_mean:.4g}; "
          f"events/pk {g.mc_steps / ng:.4g} vs {o.mc_steps_sum / no:.4g}; to_ddmc {g.to_ddmc / ng:.4g} vs "
          f"{o.to_ddmc / no:.4g}; absorbed {g.absorbed / ng:.4g} vs {o.absorbed / no:.4g}", flush=True)
    assert_spectrum_matches(r)
    se = math.sqrt(g.t_var / g.escaped + o.t_var / o.escaped)
    assert abs(g.t_mean - o.t_mean) < 4.5 * se
    for a, b in ((g.mc_steps, o.mc_steps_sum), (g.to_ddmc, o.to_ddmc), (g.to_mc, o.to_mc), (g.absorbed, o.absorbed)):
        fa, fb = a / ng, b / no
        assert abs(fa - fb) <= 6 * math.sqrt(b + 1) / no + 0.03 * max(fa, fb), (fa, fb)


def test_single_scattering_limit():
    """A slab of line-centre depth 1e-4 in its source bin: unscattered escapes E_2(tau), one
    scattering into bin j with O6's probability."""
    edges = np.array([-8.0, -5.0, -3.2, -1.0, 1.0, 3.2, 5.0, 8.0])
    m = media.slab(1.0, 1e4, 4, 7).replace(bin_edges=edges, tau_threshold=THIN, flags=G)
    tau, n = 1e-4, 1 << 26
    m = m.replace(k0=np.full(4, tau / tb.build(m).k[0, 3]), n_packets=n)
    p = rddmc.Problem(m)
    p.run(seed=4)
    g = p.results()[0]
    spec = g.spectrum.sum(axis=0)[1:-1].astype(np.float64)
    p_sc = 1.0 - special.expn(2, tau)
    row = np.array([rd.group_probability(edges, media._a_of_T(1e4), 3, j, epsrel=1e-6) for j in range(7)])
    want = n * p_sc * row
    want[3] += n * (1.0 - p_sc)
    z = (spec - want) / np.sqrt(np.maximum(n * p_sc * row * (1.0 - p_sc * row), 1.0))
    print(f"[groups] single scattering: counts {spec.astype(np.int64)}, z {np.round(z, 2)}", flush=True)
    assert g.escaped == n
    assert np.all(np.abs(z) < 4.0)


def test_group_walk_is_bit_identical_across_launch_shapes():
    m = CASES["slab_hybrid_groups"].with_packets(1 << 14)
    out = []
    for kw in (dict(), dict(block=64, grid=7, chunk=3), dict(block=256, grid=301, chunk=50)):
        p = rddmc.Problem(m)
        p.run(seed=7, **kw)
        out.append(p.tallies.cpu().numpy().copy())
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])
