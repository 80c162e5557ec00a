"""O1 (literal min-of-exponentials walker) against O2 (exact chain): the two oracles
implement the same method two independent ways."""
import math

import numpy as np
import pytest

from oracle import chain, walk
from paper_1709_10187_amd import media
from tests._stats import assert_spectrum_matches, compare_exact

CASES = {
    "slab_static": media.slab(300.0, 1e4, 8, 16, x_max=6.0),
    "sphere_outflow": media.sphere(1e3, 1e4, 8, 24, x_max=8.0, v_max=20.0),
    "slab_cold_odd_bins": media.slab(1e3, 1e2, 6, 15),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_o1_matches_o2(name):
    m = CASES[name]
    r = chain.solve(m)
    n = 60000
    w = walk.run(m, n_packets=n, seed=11)
    assert w.escaped == n and w.capped == 0
    res = compare_exact(w.spectrum, r.spectrum, n)
    assert_spectrum_matches(res, l1_max=max(0.03, 2.5 * res["expected_noise_L1"]))
    assert abs(w.steps_mean - r.steps) < 4 * math.sqrt(r.steps_var / n)
    assert abs(w.t_mean - r.t_mean) < 4 * math.sqrt(r.t_var / n)
    assert abs(w.t2_sum / n - r.t2) < 5 * math.sqrt(max(r.t2, 1e-30) ** 2 * 4 / n) + 0.05 * r.t2


def test_o1_is_deterministic_and_thread_independent():
    m = CASES["slab_static"]
    a = walk.run(m, n_packets=5000, seed=5, n_threads=1)
    b = walk.run(m, n_packets=5000, seed=5, n_threads=7)
    assert np.array_equal(a.spectrum, b.spectrum)
    assert np.array_equal(a.time_hist, b.time_hist)
    assert a.steps_sum == b.steps_sum


def test_o1_shards_sum_to_whole():
    m = CASES["slab_static"]
    whole = walk.run(m, n_packets=4000, seed=9)
    parts = [walk.run(m, n_packets=1000, seed=9, first_id=1000 * i) for i in range(4)]
    assert np.array_equal(whole.spectrum, sum(p.spectrum for p in parts))


def test_o1_step_cap_counts():
    m = CASES["slab_static"]
    w = walk.run(m, n_packets=2000, seed=1, max_steps=100)
    assert w.capped + w.escaped == 2000
    assert w.capped > 1500
    assert w.steps_max == 100
