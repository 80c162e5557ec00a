"""Pins of the oracle walker's continuous dust weights (Sec. 2.4's second method) against the
exact chain, whose dust absorption is a killing channel: the expected escaped weight per slot
is the chain's escape probability, the weighted mean escape time its mean escape time, and the
weighted 'bin' and 'path' estimators (with the path correction) are the killed chain's
transient expectations, and eq. 18's is the chain's with leak probabilities r_f / K_leak (no
absorption event ends a weighted step); and the two dust methods of the oracle walker against each other on a
hybrid slab with continuous-MC wings.  Weights lie in [0, 1], so every weighted estimator's
variance is at most its mean."""
import math

import numpy as np

from oracle import chain, walk1dh
from paper_1709_10187_amd import media
from tests._stats import assert_spectrum_matches, compare_weighted_exact, compare_weighted_two

W = media.DUST_WEIGHT


def dusty_sphere():
    m = media.sphere(400.0, 1e4, 6, 16, x_max=6.0, v_max=10.0)
    return m.replace(dust_abs=np.linspace(0.5, 2.0, 6), dust_sca=np.full(6, 3.0), flags=W)


def test_weighted_escapes_match_the_killed_chain():
    m = dusty_sphere()
    ref = chain.solve(m)
    n = 1 << 16
    o = walk1dh.run(m, n_packets=n, seed=21)
    assert o.escaped + o.absorbed == n and o.capped == 0
    r = compare_weighted_exact(o.wspec, o.wspec2, n, ref.spectrum.ravel())
    assert_spectrum_matches(r)
    esc = 1.0 - ref.absorbed
    sd = math.sqrt(max(o.wspec2.sum() / n - (o.w_sum / n) ** 2, 1e-300) / n)
    assert abs(o.w_sum / n - esc) < 4 * sd
    assert abs(o.t_mean_w - ref.t_mean) < 4.5 * math.sqrt(ref.t_var / (o.w_sum * o.w_sum / o.wspec2.sum()))
    assert o.absorbed < n // 100      # only weights below 1e-10 are dropped


def test_weighted_census_and_acceleration_match_the_killed_transient_law():
    m = media.slab(100.0, 1e4, 4, 6, x_max=4.0).replace(dust_abs=np.array([0.3, 0.8, 0.8, 0.3]),
                                                        dust_sca=np.full(4, 0.5), flags=W)
    ref = chain.solve(m)
    edges = np.array([0.0, 0.2, 0.5, 1.0, 2.0, 4.0]) * ref.t_mean
    ex = chain.transient(m, edges, dust_weights=True)
    n = 1 << 17
    o = walk1dh.run(m.replace(census=edges), n_packets=n, seed=23)
    p = ex.at_edges.ravel()
    got = o.e_bin.ravel() / n
    tol = 5 * np.sqrt(np.maximum(p, 1e-30) / n) + 1e-6
    assert np.all(np.abs(got - p) <= tol)
    dt = np.diff(edges)[:, None, None]
    mean = (o.e_path / (n * dt)).ravel()
    want = ex.mean_in.ravel()
    tol = 5 * np.sqrt(np.maximum(want, 1e-30) / n) + 1e-6
    assert np.all(np.abs(mean - want) <= tol)
    # eq. 18 with the path correction, against the chain's expectation for weighted walks (its
    # per-packet spread from eight independent seeds); the probabilistic method's expectation
    # (r_f / (K_leak + k_a) per unit residence) differs here by about 20 %
    runs = np.array([walk1dh.run(m.replace(census=edges), n_packets=1 << 15, seed=60 + b).e_accel / (1 << 15)
                     for b in range(8)])
    mean, se = runs.mean(axis=0), runs.std(axis=0, ddof=1) / math.sqrt(len(runs))
    assert np.all(np.abs(mean - ex.accel) <= 5.0 * se + 1e-9), (mean, ex.accel, se)
    other = chain.transient(m, edges).accel
    assert np.max(np.abs(other - ex.accel) / np.maximum(se, 1e-12)) > 10   # the test tells the two apart


def test_weights_and_probabilistic_absorption_agree_on_a_hybrid_slab():
    """The two dust methods estimate the same escape spectrum: continuous-MC wings, dust
    scattering and absorption in both kinds of states."""
    base = media.slab(2e4, 1e4, 12, 48, x_max=20.0, tau_threshold=10.0).replace(
        dust_abs=np.full(12, 2.0), dust_sca=np.full(12, 1.0))
    n = 1 << 14
    pr = walk1dh.run(base, n_packets=n, seed=25)
    wt = walk1dh.run(base.replace(flags=W), n_packets=n, seed=27)
    c = pr.spectrum.astype(np.float64)
    r = compare_weighted_two(wt.wspec, wt.wspec2, n, c, c, n)
    assert_spectrum_matches(r)
    assert abs(wt.w_sum / n - pr.escaped / n) < 4 * math.sqrt(pr.escaped / n / n + wt.wspec2.sum() / n / n)
