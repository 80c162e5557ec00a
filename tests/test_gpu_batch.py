"""Batched transport: many independent clouds in one persistent launch (the sweep), with
per-cloud parity against the exact chain, independence of a cloud's result from its
batch, HIP-graph replay and the launch-schedule autotuner."""
import math

import numpy as np
import pytest

from oracle import chain
from paper_1709_10187_amd import autotune, media, rddmc
from tests._stats import assert_spectrum_matches, compare_exact

pytestmark = pytest.mark.gpu


def _small_sweep():
    """Four small clouds in the style of the sweep: outflowing spheres of different depth,
    temperature, shell and bin counts and velocity."""
    spec = [(3e3, 1e4, 12, 40, 30.0), (1e3, 3e2, 9, 55, 8.0), (5e3, 2e3, 16, 33, 0.0),
            (2e3, 5e4, 7, 24, 120.0)]
    meds = []
    for tau0, T, ns, nb, vmax in spec:
        c = media.SweepCloud(tau0, T, ns, nb, vmax, 25000)
        meds.append(media.sweep_cloud_medium(c))
    return meds


def test_batch_matches_chain_per_cloud():
    meds = _small_sweep()
    p = rddmc.Problem(meds)
    p.run(seed=5)
    res = p.results()
    for m, r in zip(meds, res):
        ref = chain.solve(m)
        n = m.n_packets
        print(m.name, r.launched, r.steps_mean, ref.steps, flush=True)
        assert r.launched == r.escaped == n
        cmp = compare_exact(r.spectrum, ref.spectrum, n)
        assert_spectrum_matches(cmp, l1_max=max(0.015, 2.5 * cmp["expected_noise_L1"]))
        assert abs(r.steps_mean - ref.steps) < 4 * math.sqrt(ref.steps_var / n)
        assert abs(r.t_mean - ref.t_mean) < 4 * math.sqrt(ref.t_var / n)


def test_cloud_result_independent_of_batch():
    meds = _small_sweep()
    p = rddmc.Problem(meds, streams=[11, 12, 13, 14])
    p.run(seed=2)
    together = p.results()
    for k, m in enumerate(meds):
        q = rddmc.Problem([m], streams=[11 + k])
        q.run(seed=2, block=64, chunk=9)
        alone = q.results()[0]
        np.testing.assert_array_equal(alone.spectrum, together[k].spectrum)
        np.testing.assert_array_equal(alone.time_hist, together[k].time_hist)
        assert alone.steps_total == together[k].steps_total and alone.t_mean == together[k].t_mean


def test_graph_replay_matches_eager():
    import torch
    meds = _small_sweep()
    eager = rddmc.Problem(meds)
    eager.run(seed=7)
    ref = eager.results()
    p = rddmc.Problem(meds)
    g = p.capture(seed=7)
    torch.cuda.synchronize()
    for rep in range(3):
        p.reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = p.results()
        _ = torch.zeros(1, device="cuda").sum().item()     # eager work between replays
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a.spectrum, b.spectrum)
            np.testing.assert_array_equal(a.step_hist, b.step_hist)
            assert a.steps_total == b.steps_total and a.t_mean == b.t_mean


def test_autotuner_picks_a_working_schedule():
    meds = _small_sweep()
    p = rddmc.Problem(meds)
    best = autotune.tune(p, sample_packets=1 << 16, trial_steps=4000, use_cache=False,
                         candidates=[(64, 512, 32), (256, 1024, 128), (128, 2048, 32)],
                         tail_candidates=(16, -1, 32), tail_packets_per_cloud=256)
    assert best["steps_per_s"] > 0 and len(best["trials"]) == 3
    assert len(best["tail_trials"]) == 3 and best["tail_lanes"] in (16, -1, 32)
    print(f"[batch] autotuned {autotune.schedule(best)}; tail trials "
          f"{[(t['tail_lanes'], round(t['ms'], 1)) for t in best['tail_trials']]}", flush=True)
    p.run(seed=5, **autotune.schedule(best))
    q = rddmc.Problem(meds)
    q.run(seed=5)
    for a, b in zip(p.results(), q.results()):
        np.testing.assert_array_equal(a.spectrum, b.spectrum)


def test_longest_first_order_from_the_pilot():
    """The pilot's per-cloud cost orders the clouds; a denser cloud of the same grid walks longer."""
    base = media.slab(200.0, 1e4, 8, 16)
    meds = [base.replace(k0=np.full(8, tau)) for tau in (50.0, 800.0, 200.0)]
    cost = autotune.pilot_costs(meds, packets=256)
    assert autotune.longest_first(cost) == [1, 2, 0]


def test_sweep_clouds_at_full_grid():
    """Two clouds of the 256-cloud sweep at their full grids (outflow, cold gas), a sample of
    their packets, against the exact chain."""
    ps = media.sweep_parameters()
    meds = [media.sweep_cloud_medium(ps[i]).with_packets(2000) for i in (127, 212)]
    print("[batch] two sweep clouds at full grid, 2000 packets each", flush=True)
    p = rddmc.Problem(meds, streams=[127, 212])
    p.run(seed=0)
    res = p.results()
    print("[batch] transport done", flush=True)
    for m, r in zip(meds, res):
        ref = chain.solve(m)
        cmp = compare_exact(r.spectrum, ref.spectrum, m.n_packets)
        print(m.name, {k: v for k, v in cmp.items() if k != "z"}, flush=True)
        assert_spectrum_matches(cmp)
        assert abs(r.steps_mean - ref.steps) < 4 * math.sqrt(ref.steps_var / m.n_packets)
