"""Pins of the exact single-cell exit law (O5): the whole-medium chain on a one-cell slab,
brute-force sampling of the in-cell chain, the one-bin closed form, conservation and the
static mirror symmetry."""
import math

import numpy as np
import pytest

from oracle import chain, exitlaw
from oracle import tables as tb
from paper_1709_10187_amd import media


def test_one_cell_slab_equals_whole_medium_chain():
    """A one-cell slab: leaving the cell is escaping, so the exit law is the chain's escape
    spectrum (static media tally the exit bin) with the same step and time moments."""
    m = media.slab(400.0, 1e4, 1, 24, x_max=8.0)
    t = tb.build(m)
    for j_in in (11, 12, 3):
        src = m.replace(src_x=np.array([0.5 * (t.bin_edges[j_in] + t.bin_edges[j_in + 1])]))
        c = chain.solve(src)
        e = exitlaw.exit_law(t, 0, j_in)
        np.testing.assert_allclose(e.prob, c.spectrum[:, 1:-1], rtol=1e-9, atol=1e-15)
        assert e.steps == pytest.approx(c.steps, rel=1e-10)
        assert e.t_mean == pytest.approx(c.t_mean, rel=1e-10)
        assert e.t2 == pytest.approx(c.t2, rel=1e-9)


def test_against_brute_force_sampling_interior_moving_cell():
    """Interior cell of a moving slab (face rates use the Doppler-shifted neighbours)."""
    m = media.slab(60.0, 1e4, 3, 9, x_max=5.0, vel=np.array([-8.0, 0.0, 12.0]))
    t = tb.build(m)
    n = 200000
    counts, steps, tmean = exitlaw.simulate(t, 1, 4, n, seed=2)
    e = exitlaw.exit_law(t, 1, 4)
    assert e.prob.sum() == pytest.approx(1.0, abs=1e-12)
    p = e.prob
    sig = np.sqrt(np.maximum(p * (1 - p), 1e-300) / n)
    z = (counts / n - p) / sig
    mask = p * n >= 10
    assert np.abs(z[mask]).max() < 4.5
    assert abs(steps - e.steps) < 5 * math.sqrt(e.steps * 10 / n) + 0.01 * e.steps
    assert abs(tmean - e.t_mean) < 5 * math.sqrt(e.t_var / n)


def test_one_bin_closed_form():
    m = media.slab(50.0, 1e4, 3, 1, x_max=1.0)
    t = tb.build(m)
    e = exitlaw.exit_law(t, 1, 0)
    r = t.rate_face[1, 0]
    K = r.sum()
    np.testing.assert_allclose(e.prob[:, 0], r / K, rtol=1e-14)
    assert e.steps == pytest.approx(1.0, rel=1e-14)
    assert e.t_mean == pytest.approx(1.0 / K, rel=1e-14)
    assert e.t2 == pytest.approx(2.0 / K ** 2, rel=1e-13)


def test_static_cell_mirror_symmetry():
    m = media.slab(1e4, 1e4, 5, 31, x_max=12.0)
    t = tb.build(m)
    e = exitlaw.exit_law(t, 2, 15)
    np.testing.assert_allclose(e.prob[0], e.prob[1], rtol=1e-10)
    np.testing.assert_allclose(e.prob[0], e.prob[0][::-1], rtol=1e-8)


def test_exit_time_moments_per_bin_against_brute_force():
    """E[T | exit bin] and E[T^2 | exit bin] of the first-step recursions against brute-force
    sampling of the in-cell chain (moving interior cell)."""
    m = media.slab(60.0, 1e4, 3, 9, x_max=5.0, vel=np.array([-8.0, 0.0, 12.0]))
    t = tb.build(m)
    n = 400000
    counts, _, _, ts, t2s = exitlaw.simulate(t, 1, 4, n, seed=3, per_bin=True)
    m1, m2 = exitlaw.exit_time_moments(t, 1, 4)
    cnt = counts.sum(axis=0)
    for jo in np.nonzero(cnt >= 2000)[0]:
        mean = ts[jo] / cnt[jo]
        sec = t2s[jo] / cnt[jo]
        var = max(m2[jo] - m1[jo] ** 2, 1e-300)
        assert abs(mean - m1[jo]) < 5 * math.sqrt(var / cnt[jo]), (jo, mean, m1[jo])
        assert sec == pytest.approx(m2[jo], rel=0.1)


def test_exit_time_moments_consistent_with_the_exit_law():
    """Averaged over the exit law, the per-bin moments give exit_law's E[T] and E[T^2] (computed
    there by a different formula)."""
    m = media.sphere(3e3, 1e3, 6, 21, x_max=8.0, v_max=30.0)
    t = tb.build(m)
    for cell, j_in in ((2, 10), (4, 7)):
        e = exitlaw.exit_law(t, cell, j_in)
        m1, m2 = exitlaw.exit_time_moments(t, cell, j_in)
        pj = e.prob.sum(axis=0)
        ok = pj > 0
        assert np.sum(pj[ok] * m1[ok]) == pytest.approx(e.t_mean, rel=1e-10)
        assert np.sum(pj[ok] * m2[ok]) == pytest.approx(e.t2, rel=1e-10)


def test_exit_time_moments_one_bin_closed_form():
    m = media.slab(50.0, 1e4, 3, 1, x_max=1.0)
    t = tb.build(m)
    K = t.rate_face[1, 0].sum()
    m1, m2 = exitlaw.exit_time_moments(t, 1, 0)
    assert m1[0] == pytest.approx(1.0 / K, rel=1e-14)
    assert m2[0] == pytest.approx(2.0 / K ** 2, rel=1e-13)
