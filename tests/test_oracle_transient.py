"""Pins of the exact chain's transient law (the expectations of the time-dependent estimators
of eq. 17) and of its dust-absorption channel (Sec. 2.4): a single state's exponential decay,
the grey birth-death chain against the method-of-images Bessel closed form of the
continuous-time random walk, the time integral against the mean escape time, the emission
window against a quadrature of the flash law, and the killed gambler's ruin."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import chain
from oracle import tables as tb
from paper_1709_10187_amd import media


def _grey(N, k=50.0, **kw):
    """Grey slab of N cells (one frequency bin) whose vacuum faces leak at the interior rate
    (extrapolation distance k dz / 2): a symmetric nearest-neighbour walk absorbed at 0, N+1."""
    m = media.slab(k, 1e4, N, 1, x_max=1.0, **kw)
    dz = 2.0 / N
    kbin = float(tb.build(m).k[0, 0])
    return m.replace(lam=kbin * dz / 2.0), kbin, dz


def test_single_state_decays_exponentially():
    m = media.slab(3.0, 1e4, 1, 1, x_max=2.0, src_z=0.3)
    K = float(tb.build(m).K[0, 0])
    edges = np.array([0.0, 0.1, 0.25, 1.0, 3.0]) / K
    r = chain.transient(m, edges)
    np.testing.assert_allclose(r.at_edges[:, 0, 0], np.exp(-K * edges), rtol=1e-12)
    want = (np.exp(-K * edges[:-1]) - np.exp(-K * edges[1:])) / (K * np.diff(edges))
    np.testing.assert_allclose(r.mean_in[:, 0, 0], want, rtol=1e-11)
    np.testing.assert_allclose(r.escaped_by, 1.0 - np.exp(-K * edges), rtol=1e-11, atol=1e-15)


@pytest.mark.parametrize("N,start", [(9, 5), (15, 3)])
def test_grey_chain_against_images_of_bessel_walk(N, start):
    """Continuous-time symmetric walk with hop rate r each way started at cell m: on the
    integers P(n, t) = exp(-2rt) I_{n-m}(2rt); absorbing points at 0 and L = N + 1 give the
    image sum over k of [I_{n-m+2kL} - I_{n+m+2kL}]."""
    m, kbin, dz = _grey(N)
    zc = -1 + dz * (start - 0.5)
    m = m.replace(src_pos=np.array([[zc, 0, 0]]))
    r_hop = 1.0 / (3.0 * kbin * dz * dz)      # eq. 10 between equal cells: 2 / (3 * 2 k dz) / dz
    L = N + 1
    times = np.array([0.0, 0.3, 1.0, 4.0, 12.0]) / r_hop
    res = chain.transient(m, times)
    for it, t in enumerate(times):
        z = 2.0 * r_hop * t
        n = np.arange(1, N + 1)
        P = np.zeros(N)
        for k in range(-8, 9):
            P += special.ive(n - start + 2 * k * L, z) - special.ive(n + start + 2 * k * L, z)
        if t == 0.0:
            P = (n == start).astype(float)
        np.testing.assert_allclose(res.at_edges[it, :, 0], P, rtol=1e-9, atol=1e-13)


def test_time_integral_is_the_mean_escape_time():
    m = media.sphere(1e3, 1e4, 6, 20, x_max=8.0, v_max=15.0)
    ref = chain.solve(m)
    edges = np.array([0.0, 0.5 * ref.t_mean, 2 * ref.t_mean, 200 * ref.t_mean])
    r = chain.transient(m, edges)
    integral = float((r.mean_in.sum(axis=(1, 2)) * np.diff(edges)).sum())
    assert integral == pytest.approx(ref.t_mean, rel=1e-9)
    assert r.escaped_by[-1] == pytest.approx(1.0, abs=1e-12)
    # P(still inside at t) + P(escaped by t) = 1
    np.testing.assert_allclose(r.at_edges.sum(axis=(1, 2)) + r.escaped_by, 1.0, atol=1e-11)


def test_emission_window_is_the_averaged_flash_law():
    m = media.slab(200.0, 1e4, 4, 6, x_max=5.0)
    ts, te = 0.2, 1.7
    t = 2.5
    w = chain.transient(m, np.array([0.0, t]), emit=(ts, te))
    flash = lambda s: chain.transient(m, np.array([0.0, s])).at_edges[1] if s > 0 else chain.transient(
        m, np.array([0.0, 1e-300])).at_edges[0]
    # quadrature over the emission time of the flash occupation at t - tau
    acc = np.zeros_like(w.at_edges[1])
    nodes, wts = np.polynomial.legendre.leggauss(40)
    for x, wt in zip(nodes, wts):
        tau = ts + 0.5 * (x + 1.0) * (te - ts)
        acc += 0.5 * wt * flash(t - tau)
    np.testing.assert_allclose(w.at_edges[1], acc, rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("N,start,q", [(9, 5, 0.01), (14, 2, 0.05)])
def test_dust_absorption_is_the_killed_gamblers_ruin(N, start, q):
    """A grey walk killed with probability q per step (absorption rate k_a = q K / (1 - q)):
    the escape probability from m is cosh(theta (m - L/2)) / cosh(theta L/2) with
    cosh(theta) = 1 / (1 - q), L = N + 1; escape and absorption add to one."""
    m0, kbin, dz = _grey(N)
    K = float(tb.build(m0).K[0, 0])
    ka = q * K / (1.0 - q)
    zc = -1 + dz * (start - 0.5)
    m = m0.replace(src_pos=np.array([[zc, 0, 0]]), dust_abs=np.full(N, ka))
    r = chain.solve(m)
    L = N + 1
    th = math.acosh(1.0 / (1.0 - q))
    want = math.cosh(th * (start - L / 2.0)) / math.cosh(th * L / 2.0)
    assert r.total == pytest.approx(want, rel=1e-10)
    assert r.total + r.absorbed == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("N,start", [(9, 5), (11, 3)])
def test_acceleration_steady_grey_slab_is_the_net_face_crossings(N, start):
    """Eq. 18 over one long interval on a grey slab whose every state has the same total rate K:
    each leak across a face adds k dl along its motion to both cells it touches, E[dl] = 1/K,
    so cell i collects (k/K) times the expected net upward crossings of its two faces,
    P_top - 1{m > i} and P_top - 1{m >= i} (walk from cell m absorbed at 0 and N+1,
    P_top = m / (N+1))."""
    m0, kbin, dz = _grey(N)
    t = tb.build(m0)
    np.testing.assert_allclose(t.K[:, 0], t.K[0, 0], rtol=1e-12)
    K = float(t.K[0, 0])
    zc = -1 + dz * (start - 0.5)
    m = m0.replace(src_pos=np.array([[zc, 0, 0]]))
    t_end = 400.0 * chain.solve(m).t_mean
    r = chain.transient(m, np.array([0.0, t_end]))
    assert r.escaped_by[-1] == pytest.approx(1.0, abs=1e-12)
    p_top = start / (N + 1.0)
    i = np.arange(1, N + 1)
    want = kbin / K * (2.0 * p_top - (start > i) - (start >= i))
    np.testing.assert_allclose(r.accel[0], want, rtol=1e-9, atol=1e-12)


def test_acceleration_per_interval_against_the_bessel_walk():
    """The same estimator per census interval: cell i collects k r / K times the time integral
    of P_{i-1}(t) - P_{i+1}(t) over the interval (the hop rate r each way, P_0 = P_{N+1} = 0),
    with P from the image sum of the continuous-time walk."""
    from scipy import integrate
    N, start = 9, 4
    m0, kbin, dz = _grey(N)
    K = float(tb.build(m0).K[0, 0])
    m = m0.replace(src_pos=np.array([[-1 + dz * (start - 0.5), 0, 0]]))
    r_hop = 1.0 / (3.0 * kbin * dz * dz)
    assert K == pytest.approx(2.0 * r_hop, rel=1e-12)
    L = N + 1
    edges = np.array([0.0, 0.5, 2.0, 6.0]) / r_hop
    res = chain.transient(m, edges)

    def P(n, t):
        if n < 1 or n > N:
            return 0.0
        z = 2.0 * r_hop * t
        return sum(special.ive(n - start + 2 * k * L, z) - special.ive(n + start + 2 * k * L, z)
                   for k in range(-8, 9))

    for it in range(len(edges) - 1):
        for i in range(1, N + 1):
            val, _ = integrate.quad(lambda s: P(i - 1, s) - P(i + 1, s), edges[it], edges[it + 1],
                                    epsabs=1e-13, epsrel=1e-11, limit=200)
            assert res.accel[it, i - 1] == pytest.approx(kbin * r_hop / K * val, rel=1e-7, abs=1e-10)


def test_walker_acceleration_matches_exact_chain():
    """The literal walker's per-leak sums against the chain's expectation on a small moving
    sphere (Doppler re-binning decides the inward leak's bin): eight independent batches give
    the standard error."""
    from oracle import walk1dh
    m = media.sphere(400.0, 1e4, 4, 10, x_max=6.0, v_max=25.0)
    ref = chain.solve(m)
    edges = np.array([0.0, 0.3, 1.0, 3.0]) * ref.t_mean
    m = m.replace(census=edges)
    ex = chain.transient(m, edges).accel
    n = 1 << 14
    runs = np.array([walk1dh.run(m, n_packets=n, seed=100 + b).e_accel / n for b in range(8)])
    mean, se = runs.mean(axis=0), runs.std(axis=0, ddof=1) / math.sqrt(len(runs))
    z = np.abs(mean - ex) / np.maximum(se, 1e-12)
    print(f"walker vs chain eq. 18: max |z| {z.max():.2f}")
    assert np.all(np.abs(mean - ex) <= 5.0 * se + 1e-9 * np.abs(ex).max())
