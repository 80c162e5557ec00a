"""The paper's efficient frequency grid (Secs. 4.2 and 5.1, eq. 37): its construction, and the
exact chain on it against the analytic spectra (eq. 33 for the slab, the derived sphere
solution) next to the uniform grids the workloads use.

Bars: at a tau0 = 1e9 (T = 10 K, the paper's converged setups) the grid's spectrum lies within
L1 0.003 of the analytic one and its mean |x| within 0.2 %, with fewer DDMC steps per packet
than the uniform grids of the same setups; on the tau0 = 1e7 sphere (a tau0 = 4.7e3) it is as
close to the analytic spectrum as the 512-bin uniform grid (within 0.005 in L1, the analytic
solution's own error dominating both), with the same mean escape time (1 %) and over a
thousand times fewer steps."""
import math

import numpy as np
import pytest

from oracle import analytic as an
from oracle import chain
from paper_1709_10187_amd import media


@pytest.mark.parametrize("T", [10.0, 1.0e2, 1.0e4])
def test_core_wing_crossover_solves_its_equation(T):
    a = media._a_of_T(T)
    x = media.core_wing_crossover(a)
    assert x > 1.0
    assert math.exp(-x * x) == pytest.approx(a / (math.sqrt(math.pi) * x * x), rel=1e-12)


def test_efficient_grid_structure():
    a = media._a_of_T(1.0e4)
    xcw = media.core_wing_crossover(a)
    e = media.efficient_edges(a, 1.0e7, 1.0 / 256)
    n = len(e) - 1
    assert n % 2 == 1
    np.testing.assert_array_equal(e, -e[::-1])
    dx = np.diff(e)
    assert dx[n // 2] == pytest.approx(2.0 * xcw, rel=1e-14)         # central bin: 2 x_cw
    np.testing.assert_allclose(np.delete(dx, n // 2), 1.0, rtol=1e-12)   # eq. 37 gives 0.56: floor of 1
    xmax = 2.5 * (a * 1.0e7) ** (1.0 / 3.0)
    assert xmax <= e[-1] < xmax + 1.0
    # a wide matched wing sets the central bin too (eq. 37 with a tau0 = 1e9, dz / R = 2 / 201)
    a10 = media._a_of_T(10.0)
    e = media.efficient_edges(a10, 1.0e9 / a10, 2.0 / 201)
    dxw = (2.5 * 1.0e9 * (2.0 / 201) ** 2) ** (1.0 / 3.0)
    np.testing.assert_allclose(np.diff(e), dxw, rtol=1e-12)
    assert (len(e) - 1) % 2 == 1


def _spec(r):
    s = r.spectrum
    s = s.sum(axis=0) if s.ndim == 2 else s
    s = s[1:-1]
    return s / s.sum()


def _against_analytic(m, pdf, atau):
    r = chain.solve(m)
    p = _spec(r)
    q = an.binned(pdf, m.bin_edges, atau)
    q = q / q.sum()
    c = 0.5 * (m.bin_edges[1:] + m.bin_edges[:-1])
    return r, float(np.abs(p - q).sum()), float(np.sum(p * np.abs(c))), float(np.sum(q * np.abs(c)))


@pytest.mark.parametrize("geo", ["slab", "sphere"])
def test_efficient_grid_on_the_converged_setups(geo):
    a = media._a_of_T(10.0)
    tau0 = 1.0e9 / a
    base = media.validation_slab() if geo == "slab" else media.validation_sphere()
    dz = 2.0 / 201 if geo == "slab" else 1.0 / 200
    pdf = an.slab_pdf if geo == "slab" else an.sphere_pdf
    eff = base.replace(bin_edges=media.efficient_edges(a, tau0, dz))
    ru, l1u, _, _ = _against_analytic(base, pdf, 1.0e9)
    re, l1e, xe, xq = _against_analytic(eff, pdf, 1.0e9)
    print(f"{geo}: uniform {base.n_bins} bins L1 {l1u:.4f} steps {ru.steps:.4g}; efficient {eff.n_bins} bins "
          f"L1 {l1e:.4f} steps {re.steps:.4g}; <|x|> {xe:.2f} vs {xq:.2f}")
    assert l1e < 0.003
    assert xe == pytest.approx(xq, rel=0.002)
    assert re.steps < ru.steps
    assert re.t_mean == pytest.approx(ru.t_mean, rel=0.01)


def test_efficient_grid_on_the_tau1e7_sphere():
    a = media._a_of_T(1.0e4)
    base = media.config_sphere()
    eff = base.replace(bin_edges=media.efficient_edges(a, 1.0e7, 1.0 / 256))
    ru, l1u, _, _ = _against_analytic(base, an.sphere_pdf, a * 1.0e7)
    re, l1e, _, _ = _against_analytic(eff, an.sphere_pdf, a * 1.0e7)
    print(f"tau0 1e7 sphere: uniform L1 {l1u:.4f} steps {ru.steps:.4g}; efficient {eff.n_bins} bins L1 {l1e:.4f} "
          f"steps {re.steps:.4g}")
    assert l1e < l1u + 0.005
    assert re.t_mean == pytest.approx(ru.t_mean, rel=0.01)
    assert ru.steps / re.steps > 1000.0
