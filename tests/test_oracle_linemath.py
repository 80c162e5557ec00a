"""Pins of the oracle's line physics (eqs. 12-14) against independent mathematics."""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

from oracle import linemath as lm


@pytest.mark.parametrize("x", [0.0, 1e-3, 0.2, 0.7, 1.5, 3.0, 7.0, 25.0, 400.0])
def test_dawson_against_mpmath(x):
    # F(x) = sqrt(pi)/2 exp(-x^2) erfi(x)
    mpmath.mp.dps = 40
    ref = float(mpmath.sqrt(mpmath.pi) / 2 * mpmath.exp(-mpmath.mpf(x) ** 2) * mpmath.erfi(x))
    assert special.dawsn(x) == pytest.approx(ref, rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("a", [4.702e-4, 1.4869e-2])
@pytest.mark.parametrize("x", [0.05, 0.5, 1.2, 2.9, 4.0, 11.0, 60.0])
def test_Hcal_is_integral_of_H(a, x):
    """Eq. (13) must be the integral of eq. (12) from 0 to x (mpmath quadrature of eq. 12)."""
    mpmath.mp.dps = 30
    A = mpmath.mpf(a)

    def H(y):
        F = mpmath.sqrt(mpmath.pi) / 2 * mpmath.exp(-y * y) * mpmath.erfi(y)
        e = mpmath.exp(-y * y)
        return e + 2 * A / mpmath.sqrt(mpmath.pi) * (2 * y * F - 1) + A * A * e * (1 - 2 * y * y)

    pts = [0, min(x, 3.0), x] if x > 3.0 else [0, x]
    ref = float(mpmath.quad(H, pts))
    assert float(lm.voigt_Hcal(a, x)) == pytest.approx(ref, rel=1e-12, abs=1e-16)


@pytest.mark.parametrize("a", [1.5e-4, 4.702e-4, 4.7e-3, 1.4869e-2])
def test_H_expansion_against_exact_voigt(a):
    """Eq. (12) is a second-order expansion in a of the Hjerting-Voigt function
    (eq. 2), whose exact value is Re w(x + i a) (Faddeeva function)."""
    x = np.array([0.0, 0.3, 1.0, 2.0, 2.5, 3.0, 3.5, 4.0, 6.0, 10.0, 30.0, 100.0, 1000.0])
    exact = special.wofz(x + 1j * a).real
    rel = np.abs(lm.voigt_H(a, x) / exact - 1.0)
    assert rel.max() < 0.5 * a * a
    # and it is not exact: the expansion error is visible at the a^2 level
    assert rel.max() > 1e-3 * a * a


def test_H_limits():
    """Core and wing limits of eq. (2)."""
    a = 4.702e-4
    assert lm.voigt_H(a, 0.1) == pytest.approx(math.exp(-0.01), rel=2 * a)
    x = 200.0
    assert lm.voigt_H(a, x) == pytest.approx(a / (math.sqrt(math.pi) * x * x), rel=1e-3)


@pytest.mark.parametrize("a", [4.702e-4, 1.4869e-2])
@pytest.mark.parametrize("lo,hi", [(-0.3, 0.3), (0.0, 0.34), (2.8, 3.2), (3.1, 3.4), (20.0, 20.34),
                                   (-21.7, -21.3), (-0.5, 1.7), (900.0, 925.0), (-4.5, -3.9)])
def test_bin_opacity_against_quadrature(a, lo, hi):
    """Eq. (14): tophat average of k0 H over the bin, checked by direct quadrature of eq. (12)."""
    k0 = 3125.0
    pts = [p for p in (-3.0, 0.0, 3.0) if lo < p < hi]
    val, _ = integrate.quad(lambda y: float(lm.voigt_H(a, y)), lo, hi, points=pts or None,
                            epsabs=0, epsrel=1e-13, limit=200)
    assert float(lm.bin_opacity(k0, a, lo, hi)) == pytest.approx(k0 * val / (hi - lo), rel=1e-11)


def test_damping_and_thermal_velocity():
    assert float(lm.damping(1e4)) == pytest.approx(4.702e-4)
    assert float(lm.v_thermal(1e4)) == pytest.approx(12.85)
    assert float(lm.damping(10.0)) == pytest.approx(4.702e-4 * math.sqrt(1e3))


def test_core_wing_crossover():
    """x_cw solves exp(-x^2) = a / (sqrt(pi) x^2) (Sec. 2.1); at 10 K the paper quotes
    2 x_cw ~= 5 for the efficiency barrier (Sec. 4.2)."""
    for T in (10.0, 1e2, 1e4, 1e5):
        a = float(lm.damping(T))
        x = lm.x_core_wing(a)
        assert math.exp(-x * x) == pytest.approx(a / (math.sqrt(math.pi) * x * x), rel=1e-10)
    assert 2 * lm.x_core_wing(float(lm.damping(10.0))) == pytest.approx(5.0, abs=0.25)
