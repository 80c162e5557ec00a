"""Pins of O6, the discrete frequency redistribution oracle (Sec. 5.3 eq. 42, Appendix A),
against what the mathematics and the paper fix: the normalisation of the redistribution
function (its integral over the outgoing frequency against the Voigt function from the
Faddeeva routine), its a -> 0 limit and its wing limit printed in Appendix A, the wing drift
and spread quoted in Sec. 4.3 (<dx> -> -1/x, <dx^2> -> 1), the symmetry of the joint
redistribution, and the brute-force law of single scatterings (atom velocities sampled, eq. 41)
against the bin-averaged probabilities of eq. 42."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import redistribution as rd

A_LYA = 4.7e-4       # T = 1e4 K


@pytest.mark.parametrize("a", [A_LYA, 0.05])
@pytest.mark.parametrize("xp", [0.0, 1.3, 4.0, 12.0])
def test_redistribution_is_normalised_over_the_outgoing_frequency(a, xp):
    assert rd.outgoing_integral(-math.inf, math.inf, xp, a) == pytest.approx(1.0, abs=1e-9)


def test_doppler_limit_matches_the_printed_core_form():
    """a -> 0: R_II-A -> (sqrt(pi) / 2) exp(xp^2) erfc(max(|x|, |xp|)); the damping wing adds a
    relative correction of order a exp(max(|x|, |xp|)^2)."""
    a = 1e-8
    for xp in (0.0, 0.4, 1.1, 2.2):
        for x in (-2.5, -0.3, 0.35, 1.0, 3.0):
            m = max(abs(x), abs(xp))
            assert rd.r2a(x, xp, a) == pytest.approx(rd.r1a(x, xp), rel=100 * a * math.exp(m * m)), (x, xp)


def test_wing_limit_matches_the_printed_wing_form():
    """|x + xp| -> inf: the relative difference to the printed wing form falls like 1/xp^2."""
    prev = None
    for xp in (10.0, 20.0, 40.0):
        err = max(abs(rd.r2a(xp + d, xp, A_LYA) / rd.r2a_wing(xp + d, xp) - 1.0) for d in (-1.5, -0.5, 0.3, 1.2))
        assert err < 2.0 / xp ** 2, (xp, err)
        if prev is not None:
            assert err < prev / 3.0
        prev = err


@pytest.mark.parametrize("xp", [10.0, 20.0, 40.0])
def test_wing_drift_and_spread(xp):
    """Sec. 4.3: in the wing a scattering moves x by <dx> ~ -1/x with <dx^2> ~ 1."""
    m1 = integrate.quad(lambda x: (x - xp) * rd.r2a(x, xp, A_LYA), xp - 30, xp + 30, points=[xp], limit=400)[0]
    m2 = integrate.quad(lambda x: (x - xp) ** 2 * rd.r2a(x, xp, A_LYA), xp - 30, xp + 30, points=[xp], limit=400)[0]
    assert abs(m1 * xp + 1.0) < 2.5 / xp ** 2
    assert abs(m2 - 1.0) < 3.0 / xp ** 2


@pytest.mark.parametrize("a", [A_LYA, 0.05])
def test_joint_redistribution_is_symmetric(a):
    """H(xp) R(x | xp) is Hummer's symmetric joint function (the paper's footnote convention)."""
    for xp, x in ((0.3, 1.7), (2.0, -1.0), (5.0, 4.2)):
        lhs = rd.voigt_H(a, xp) * rd.r2a(x, xp, a)
        rhs = rd.voigt_H(a, x) * rd.r2a(xp, x, a)
        assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("jp", [3, 5])
def test_bin_probabilities_match_brute_force_scatterings(jp):
    """Eq. 42 (times the outgoing width) against 10^6 simulated scatterings of packets with x
    uniform in bin jp: a chi-square test over the outgoing bins, edge bins open."""
    edges = np.array([-8.0, -5.0, -3.2, -1.0, 1.0, 3.2, 5.0, 8.0])
    p = np.array([rd.group_probability(edges, A_LYA, jp, j, epsrel=1e-6) for j in range(len(edges) - 1)])
    assert p.sum() == pytest.approx(1.0, abs=1e-7)
    n = 1_000_000
    got = np.bincount(rd.sample_group(edges, A_LYA, jp, n, np.random.default_rng(11 + jp)), minlength=len(p))
    keep = p * n > 20
    exp_c = p[keep] * n
    chi2 = float(((got[keep] - exp_c) ** 2 / exp_c).sum())
    pval = stats.chi2.sf(chi2, int(keep.sum()) - 1)
    assert pval > 1e-3, (got, p * n, chi2)
    assert got[~keep].sum() <= max(10, 5 * p[~keep].sum() * n)
