"""Pins of the closed-form spectra against the paper's printed values and the mode sums."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import analytic as an

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("atau0", [47.02, 1e6, 1e9])
def test_neufeld_normalisation(atau0):
    """Eq. (33) is normalised to 1/(4 pi) (text after eq. 33)."""
    s = atau0 ** (1 / 3)
    val, _ = integrate.quad(lambda y: float(an.neufeld_J(y * s, atau0)) * s, -12, 12, limit=400,
                            epsabs=0, epsrel=1e-12)
    assert val == pytest.approx(1 / (4 * math.pi), rel=1e-9)


def test_neufeld_printed_peak_and_height():
    g = _gold("neufeld_slab.json")
    atau0 = 1e9
    s = atau0 ** (1 / 3)
    # numerical maximum of eq. (33)
    xp = optimize.minimize_scalar(lambda y: -float(an.neufeld_J(y * s, atau0)) * s, bounds=(0.5, 2.0),
                                  method="bounded", options={"xatol": 1e-11}).x
    assert xp == pytest.approx(g["peak_over_atau13"], abs=6e-5)
    height = 100 * float(an.neufeld_J(xp * s, atau0)) * s
    assert height == pytest.approx(g["peak_height_1e2_times_atau13"], abs=6e-5)
    # the printed transcendental relation xbar tanh xbar = 2/3 locates the same peak
    xbar = optimize.brentq(lambda b: b * math.tanh(b) - g["xbar_tanh_xbar"], 0.1, 3.0, xtol=1e-14)
    x_root = (xbar * atau0 / an.C_SLAB) ** (1 / 3) / s
    assert x_root == pytest.approx(xp, abs=1e-6)


@pytest.mark.parametrize("xt", [0.05, 0.3, 1.0, 2.5])
def test_slab_mode_sum_gives_eq33(xt):
    """Summing the slab's cos((n+1/2) pi z) modes gives sech(pi x~/2)/2, i.e. the shape of
    eq. (33) with pi x~/2 = sqrt(pi^3/54) x^3/(a tau0)."""
    assert an.slab_mode_sum(xt) == pytest.approx(0.5 / math.cosh(0.5 * math.pi * xt), rel=1e-12)
    assert 0.5 * math.pi * math.sqrt(2 * math.pi / 27) == pytest.approx(an.C_SLAB, rel=1e-14)


@pytest.mark.parametrize("xt", [0.05, 0.3, 1.0, 2.5])
def test_sphere_mode_sum(xt):
    assert an.sphere_mode_sum(xt) == pytest.approx(1 / (2 * (1 + math.cosh(math.pi * xt))), rel=1e-12)
    assert math.pi * math.sqrt(2 * math.pi / 27) == pytest.approx(an.C_SPHERE, rel=1e-14)


def test_wing_variable_against_printed_moments():
    """The wing variable x~ of eq. (28) fixes the steady-state profile at R (eq. 29) whose
    printed moments pin sqrt(2 pi / 27), the constant the sphere spectrum uses."""
    g = _gold("steady_state_moments.json")
    c = math.sqrt(2 * math.pi / 27)
    prof = lambda y: 1.0 / (1.0 + (c * y ** 3) ** 2)
    z, _ = integrate.quad(prof, -np.inf, np.inf)
    m1, _ = integrate.quad(lambda y: abs(y) * prof(y), -np.inf, np.inf)
    m2, _ = integrate.quad(lambda y: y * y * prof(y), -np.inf, np.inf)
    assert m1 / z == pytest.approx(g["abs_mean_over_atau13"], abs=6e-5)
    assert math.sqrt(m2 / z) == pytest.approx(g["std_over_atau13"], abs=6e-5)


def test_sphere_pdf_normalised_and_peak():
    atau0 = 1e9
    s = atau0 ** (1 / 3)
    val, _ = integrate.quad(lambda y: float(an.sphere_pdf(y * s, atau0)) * s, -12, 12, limit=400)
    assert val == pytest.approx(1.0, rel=1e-9)
    xp = optimize.minimize_scalar(lambda y: -float(an.sphere_pdf(y * s, atau0)), bounds=(0.5, 1.5),
                                  method="bounded", options={"xatol": 1e-10}).x
    # stationary point of x^2/(1+cosh(c x^3)): 2 (1 + cosh u) = 3 u sinh u, u = c x^3
    u = an.C_SPHERE * xp ** 3
    assert 2 * (1 + math.cosh(u)) == pytest.approx(3 * u * math.sinh(u), rel=1e-6)


def test_grey_chain_closed_forms():
    assert an.grey_steps(9, 5) == 25
    assert an.grey_right_exit(9, 5) == pytest.approx(0.5)
