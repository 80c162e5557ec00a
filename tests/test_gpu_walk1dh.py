"""GPU hybrid walk on 1D grids (slab planes, spherical shells) against the 1D hybrid oracle
walker (O1-1DH): escape spectra as two samples (the 3 sigma rule), mean escape times within
their noise, conversion counts; pure mode against the exact chain; the workloads of the slab,
the sphere and the sweep with continuous-MC states at tau_th = 10."""
import math

import numpy as np
import pytest

from oracle import chain, walk1dh
from paper_1709_10187_amd import media, rddmc
from tests._stats import assert_spectrum_matches, compare_exact, compare_two_samples, run_watched

pytestmark = pytest.mark.gpu

CASES = {
    "slab_all_mc": media.slab(4e2, 1e4, 16, 64, x_max=20.0, tau_threshold=1e30),
    "slab_hybrid": media.slab(2e4, 1e4, 16, 64, x_max=20.0, tau_threshold=10.0),
    "slab_hybrid_moving": media.slab(2e4, 1e4, 16, 64, x_max=20.0, tau_threshold=10.0,
                                     vel=np.linspace(-40, 40, 16)),
    "slab_hybrid_nonuniform_hot_cold": media.slab(2e4, 1e4, 16, 64, x_max=20.0, tau_threshold=5.0).replace(
        k0=2e4 * np.exp(np.sin(np.arange(16) * 1.3)), temp=1e4 * np.exp(0.5 * np.cos(np.arange(16) * 0.7))),
    "sphere_all_mc": media.sphere(3e2, 1e4, 12, 48, x_max=16.0, tau_threshold=1e30),
    "sphere_hybrid": media.sphere(3e4, 1e4, 24, 96, x_max=24.0, tau_threshold=10.0),
    "sphere_hybrid_outflow": media.sphere(3e4, 1e3, 24, 96, x_max=40.0, tau_threshold=10.0, v_max=60.0),
    "sphere_hybrid_inflow_cold": media.sphere(1e4, 1e2, 20, 121, x_max=30.0, tau_threshold=10.0, v_max=-15.0),
    "slab_core_skipping": media.slab(2e3, 1e4, 8, 32, x_max=12.0, tau_threshold=1e30).replace(x_crit=2.0),
}


def _gpu(m, n, seed=1, **kw):
    print(f"[walk1dh] {m.name} cells={m.n_cells[0]} bins={m.n_bins} tau_th={m.tau_threshold} packets={n} {kw}",
          flush=True)
    p = rddmc.Problem(m.with_packets(n))
    p.run(seed=seed, **kw)
    return p.results()[0]


@pytest.mark.parametrize("name", sorted(CASES))
def test_hybrid_walk_matches_oracle_walker(name):
    m = CASES[name]
    ng, no = 1 << 17, 1 << 14
    g = _gpu(m, ng)
    o = walk1dh.run(m, n_packets=no, seed=5)
    assert g.launched == ng and g.escaped == ng and g.capped == 0
    assert o.escaped == no
    r = compare_two_samples(g.spectrum, o.spectrum)
    print(f"    L1 {r['L1']:.4f} max|z| {r['max_abs_z']:.2f} p {r['p_value']:.3g}; t {g.t_mean:.4g} vs {o.t_mean:.4g}; "
          f"to_mc {g.to_mc / ng:.4g} vs {o.to_mc / no:.4g}, refl {g.reflected / ng:.4g} vs {o.reflected / no:.4g}",
          flush=True)
    assert_spectrum_matches(r)
    se = math.sqrt(g.t_var / ng + o.t_var / no)
    assert abs(g.t_mean - o.t_mean) < 4.5 * se
    for a, b in ((g.to_mc, o.to_mc), (g.to_ddmc, o.to_ddmc), (g.reflected, o.reflected), (g.mc_steps, o.mc_steps_sum)):
        fa, fb = a / ng, b / no
        # per-packet counts are heavy-tailed: 6 sigma of a Poisson count of the oracle sample plus 3 %
        assert abs(fa - fb) <= 6 * math.sqrt((b + 1)) / no + 0.03 * max(fa, fb), (fa, fb)


@pytest.mark.parametrize("m", [media.slab(300.0, 1e4, 2, 8, x_max=2.0),
                               media.sphere(600.0, 1e4, 3, 10, x_max=2.0, v_max=20.0)],
                         ids=["slab", "sphere_outflow"])
def test_hybrid_walk_in_pure_mode_matches_exact_chain(m):
    """A batch with a cloud at tau_th > 0 takes the hybrid walk; with every state thick
    (tau_th = 2 on grids whose every state is thicker) it must give the pure chain's law."""
    m = m.replace(tau_threshold=2.0)
    from oracle import tables as tb
    assert tb.build(m).thick.all()
    n = 100003
    g = _gpu(m, n, seed=3)
    ref = chain.solve(m.replace(tau_threshold=0.0))
    assert g.to_mc == 0 and g.escaped == n
    r = compare_exact(g.spectrum, ref.spectrum, n)
    assert_spectrum_matches(r, l1_max=max(0.01, 2.5 * r["expected_noise_L1"]))
    assert abs(g.steps_mean - ref.steps) < 4 * math.sqrt(ref.steps_var / n)
    assert abs(g.t_mean - ref.t_mean) < 4 * math.sqrt(ref.t_var / n)


def test_hybrid_bit_identical_across_launch_shapes_and_shards():
    m = CASES["sphere_hybrid_outflow"].with_packets(30000)
    out = []
    for kw in (dict(), dict(block=64, grid=7, chunk=5), dict(block=128, grid=333, chunk=200)):
        p = rddmc.Problem(m)
        p.run(seed=11, **kw)
        out.append(p.tallies.cpu().numpy().copy())
    p = rddmc.Problem(m)
    for first, count in ((0, 7000), (7000, 13), (7013, 22987)):
        p.run(seed=11, first=first, count=count, block=192, chunk=33)
    out.append(p.tallies.cpu().numpy().copy())
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])


@pytest.mark.parametrize("name", ["slab", "sphere"])
def test_workloads_at_tau_threshold_10(name):
    """The slab (tau0 = 1e5, 64 x 128) and the sphere (tau0 = 1e7, 256 x 512) at their full grids
    with continuous-MC states below tau = 10, the GPU on a packet sample against the oracle
    walker on a smaller one (the sphere's 2e7 hybrid steps per packet limit the oracle to 64 packets,
    a weak but exact-in-law two-sample test).  In the sphere every state beyond |x| ~ 3 is thin,
    so the escaping spectrum is carried by MC packets: its distance to the pure chain is the
    method's own difference, printed, not gated."""
    if name == "slab":
        m = media.config_slab().replace(tau_threshold=10.0)
        ng, no = 1 << 16, 1 << 11
    else:
        m = media.config_sphere().replace(tau_threshold=10.0)
        ng, no = 1 << 12, 1 << 6
    print(f"[walk1dh] {m.name} cells={m.n_cells[0]} bins={m.n_bins} tau_th={m.tau_threshold} packets={ng}", flush=True)
    p = rddmc.Problem(m.with_packets(ng))
    run_watched(p, seed=2, label="GPU: ")
    g = p.results()[0]
    print(f"    GPU walk done: {g.steps_mean:.4g} steps per packet; oracle walker on {no} packets", flush=True)
    spec, esc, to_mc = 0, 0, 0
    for k in range(4):   # the oracle in four runs of consecutive ids, so that progress shows
        o = walk1dh.run(m, n_packets=no // 4, seed=8, first_id=k * (no // 4))
        spec, esc, to_mc = spec + o.spectrum, esc + o.escaped, to_mc + o.to_mc
        print(f"    oracle packets {(k + 1) * (no // 4)} of {no} done", flush=True)
    assert g.escaped == ng and esc == no and g.to_mc > 0
    r = compare_two_samples(g.spectrum, spec)
    print(f"    L1 {r['L1']:.4f} max|z| {r['max_abs_z']:.2f}; to_mc/pk {g.to_mc / ng:.3g} vs {to_mc / no:.3g}",
          flush=True)
    assert_spectrum_matches(r)
    if name == "sphere":
        print("    solving the exact chain of the pure sphere", flush=True)
        ref = chain.solve(media.config_sphere())
        rp = compare_exact(g.spectrum, ref.spectrum, ng)
        print(f"    hybrid against the pure chain: L1 {rp['L1']:.4f} (noise {rp['expected_noise_L1']:.4f}), "
              f"max |z| {rp['max_abs_z']:.2f}", flush=True)


def test_sweep_clouds_at_tau_threshold_10():
    """Moving sweep clouds with continuous-MC states, as one batch, against the oracle walker
    cloud by cloud: sweep clouds 0, 32 and 56 (tau0 1.3e4-2.7e4, 44-119 shells, 27-154 km/s
    outflows), which the oracle walks at ~1e5 steps per packet."""
    params = media.sweep_parameters()
    ids = [0, 32, 56]
    meds = [media.sweep_cloud_medium(params[i], tau_threshold=10.0).with_packets(1 << 15) for i in ids]
    p = rddmc.Problem(meds, streams=ids)
    print(f"[walk1dh] sweep clouds {ids} at tau_th = 10", flush=True)
    p.run(seed=4)
    res = p.results()
    for i, m, g in zip(ids, meds, res):
        o = walk1dh.run(m, n_packets=1 << 13, seed=6)
        r = compare_two_samples(g.spectrum, o.spectrum)
        print(f"    cloud {i}: tau0 {params[i].tau0:.3g} T {params[i].T:.3g} vmax {params[i].v_max:.3g}: "
              f"max|z| {r['max_abs_z']:.2f}, to_mc/pk {g.to_mc / m.n_packets:.3g}", flush=True)
        assert g.escaped == m.n_packets
        assert_spectrum_matches(r)
