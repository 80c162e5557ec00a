"""Pins of O2 (the exact pure-DDMC chain) against analytic solutions, closed forms and
brute force on tiny inputs."""
import json
import math
import os

import numpy as np
import pytest

from oracle import analytic as an
from oracle import chain
from oracle import linemath as lm
from oracle import tables as tb
from paper_1709_10187_amd import media


def _atau0(m):
    return float(lm.damping(m.temp[0]) * m.k0[0])


def test_validation_slab_matches_neufeld():
    """The paper's converged slab (a tau0 = 1e9, T = 10 K, dz ~ 0.01 R) agrees with eq. (33)
    (Fig. 2 and Sec. 3.2.1); the chain is the noise-free limit of that run."""
    m = media.validation_slab()
    r = chain.solve(m)
    p = r.spectrum_total()[1:-1]
    ref = an.binned(an.slab_pdf, m.bin_edges, _atau0(m))
    assert abs(r.total - 1) < 1e-9
    assert np.abs(p - ref).sum() < 4e-3
    s = _atau0(m) ** (1 / 3)
    centres = 0.5 * (m.bin_edges[1:] + m.bin_edges[:-1]) / s
    assert abs(abs(centres[np.argmax(p)]) - 1.0664) < 0.06


def test_validation_sphere_matches_derived_spectrum():
    m = media.validation_sphere()
    r = chain.solve(m)
    p = r.spectrum_total()[1:-1]
    ref = an.binned(an.sphere_pdf, m.bin_edges, _atau0(m))
    assert abs(r.total - 1) < 1e-9
    assert np.abs(p - ref).sum() < 4e-3


def test_config_slab_regression_values():
    """Conservation and static symmetry of the 64x128 slab (exact properties), and its
    expected work against the stored regression values (tests/golden/chain_regression.json,
    written by make_chain_regression.py from this oracle: a guard against unintended changes,
    not a pin)."""
    m = media.config_slab()
    r = chain.solve(m)
    p = r.spectrum_total()
    assert abs(r.total - 1) < 1e-8
    assert p[0] == 0 and p[-1] == 0
    np.testing.assert_allclose(p[1:-1], p[1:-1][::-1], atol=1e-12)
    np.testing.assert_allclose(r.spectrum[0], r.spectrum[1], atol=1e-12)   # equal face fractions
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "chain_regression.json")))
    ref = g["slab_tau1e5_64x128"]
    for k in ("steps", "steps2", "t_mean", "t2"):
        assert getattr(r, k) == pytest.approx(ref[k], rel=1e-9), k


def _grey(N, k=50.0):
    """Grey slab of N cells (one frequency bin), with the extrapolation distance set to
    k dz / 2 so that the vacuum faces leak at the interior rate: a symmetric random walk
    absorbed at 0 and N+1."""
    m = media.slab(k, 1e4, N, 1, x_max=1.0)
    dz = 2.0 / N
    kbin = float(tb.build(m).k[0, 0])
    return m.replace(lam=kbin * dz / 2.0), kbin, dz


@pytest.mark.parametrize("N,start", [(9, 5), (9, 2), (16, 3), (33, 17)])
def test_grey_gamblers_ruin(N, start):
    m, kbin, dz = _grey(N)
    zc = -1 + dz * (start - 0.5)
    m = m.replace(src_pos=np.array([[zc, 0, 0]]))
    r = chain.solve(m)
    assert r.steps == pytest.approx(an.grey_steps(N, start), rel=1e-10)
    assert r.steps_var == pytest.approx(an.grey_steps_var(N, start), rel=1e-8)
    assert r.spectrum[1].sum() == pytest.approx(an.grey_right_exit(N, start), rel=1e-10)
    K = 2 / (3 * kbin * dz * dz)
    assert r.t_mean == pytest.approx(an.grey_steps(N, start) / K, rel=1e-10)


def test_single_state_time_moments():
    """One cell, one bin: the escape time is exponential with rate K, E[T^2] = 2/K^2."""
    m = media.slab(3.0, 1e4, 1, 1, x_max=2.0, src_z=0.3)
    t = tb.build(m)
    K = float(t.K[0, 0])
    r = chain.solve(m)
    assert r.steps == pytest.approx(1.0)
    assert r.t_mean == pytest.approx(1 / K, rel=1e-12)
    assert r.t2 == pytest.approx(2 / K ** 2, rel=1e-12)


def test_brute_force_tiny_chain():
    """Escape spectrum, mean steps and time moments of a 3x4-state chain against an
    explicit Neumann series sum_n P^n and a direct Monte Carlo of the jump chain."""
    m = media.slab(30.0, 1e4, 3, 4, x_max=3.0, src_z=-0.2, src_x=0.4)
    t = tb.build(m)
    r = chain.solve(m)
    nc, nb = 3, 4
    ns = nc * nb
    K = t.K.reshape(ns)
    P = np.zeros((ns, ns))
    E = np.zeros((ns, 2 * nb))
    for c in range(nc):
        for j in range(nb):
            s = c * nb + j
            if j > 0:
                P[s, s - 1] = t.rate_dn[c, j] / K[s]
            if j < nb - 1:
                P[s, s + 1] = t.rate_up[c, j] / K[s]
            for f in range(2):
                n = t.nbr[c, f]
                if n >= 0:
                    P[s, n * nb + j] += t.rate_face[c, j, f] / K[s]
                else:
                    E[s, f * nb + j] += t.rate_face[c, j, f] / K[s]
    pi0 = np.zeros(ns)
    for st, pr in tb.locate_sources(m):
        pi0[st] += pr
    acc = np.zeros(ns)
    v = pi0.copy()
    for _ in range(20000):
        acc += v
        v = v @ P
    assert np.abs(v).sum() < 1e-12
    spec = acc @ E
    assert r.steps == pytest.approx(acc.sum(), rel=1e-9)
    np.testing.assert_allclose(r.spectrum[:, 1:-1].ravel(), spec, rtol=1e-9, atol=1e-15)
    assert r.t_mean == pytest.approx(acc @ (1 / K), rel=1e-9)
    # the law of the step count N, enumerated: P(N = n) = pi0 P^(n-1) (1 - P 1)
    leave = 1.0 - P.sum(axis=1)
    v = pi0.copy()
    en1 = en2 = mass = 0.0
    for n_ in range(1, 40000):
        pn = float(v @ leave)
        mass += pn
        en1 += n_ * pn
        en2 += n_ * n_ * pn
        v = v @ P
    assert mass == pytest.approx(1.0, abs=1e-12)
    assert r.steps == pytest.approx(en1, rel=1e-9)
    assert r.steps2 == pytest.approx(en2, rel=1e-9)
    # Monte Carlo of the jump chain for E[T^2] and E[N^2]
    rng = np.random.default_rng(7)
    cum = np.cumsum(np.hstack([P, E]), axis=1)
    n = 40000
    T = np.zeros(n)
    N = np.zeros(n)
    for i in range(n):
        s = rng.choice(ns, p=pi0)
        while True:
            T[i] += rng.exponential(1 / K[s])
            N[i] += 1
            nxt = int(np.searchsorted(cum[s], rng.random(), side="right"))
            if nxt >= ns:
                break
            s = nxt
    seN = (N ** 2).std() / math.sqrt(n)
    assert abs((N ** 2).mean() - r.steps2) < 4 * seN
    se = T.std() / math.sqrt(n)
    assert abs(T.mean() - r.t_mean) < 4 * se
    se2 = (T ** 2).std() / math.sqrt(n)
    assert abs((T ** 2).mean() - r.t2) < 4 * se2


def test_velocity_mirror_and_conservation():
    """Inflow mirrors the spectrum of outflow (x -> -x) exactly, and escape probabilities
    still sum to one with Doppler re-binning."""
    out = media.sphere(1e5, 1e4, 24, 64, x_max=24.4, v_max=30.0)
    inn = out.replace(vel=-out.vel)
    ro = chain.solve(out)
    ri = chain.solve(inn)
    assert abs(ro.total - 1) < 1e-9 and abs(ri.total - 1) < 1e-9
    po, pi = ro.spectrum_total(), ri.spectrum_total()
    np.testing.assert_allclose(po, pi[::-1], atol=1e-12)
    # outflow: more flux on the red side
    mid = len(po) // 2
    assert po[:mid + 1].sum() > 0.9


def test_lab_bin_probs_is_a_distribution():
    e = np.linspace(-5, 5, 11)
    for u in (-2.3, -0.1, 0.0, 0.7, 4.0):
        p = chain.lab_bin_probs(e, 0.0, 1.0, u)
        assert p.sum() == pytest.approx(1.0, rel=1e-13)
        assert np.all(p >= -1e-15)
    # u = 0.7: mean of x + mu u is 0.5 + 0.35
    p = chain.lab_bin_probs(np.linspace(-1, 3, 401), 0.0, 1.0, 0.7)[1:-1]
    c = np.linspace(-1, 3, 401)
    cen = 0.5 * (c[1:] + c[:-1])
    assert (p * cen).sum() == pytest.approx(0.85, abs=1e-4)
