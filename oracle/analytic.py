"""Closed-form results -- oracle, test infrastructure only.

* Neufeld / Harrington slab escape spectrum, eq. (33), normalised to 1/(4 pi).
* Sphere escape spectrum: the paper prints no sphere solution.  It follows from
  the steady state of eq. (25) with the wing variable of eq. (28): with
  E = u(r, x~)/r the modes are sin(n pi r) exp(-n pi |x~|), the surface flux is
  sum_n (-1)^{n+1} n exp(-n pi |x~|) = 1 / (2 (1 + cosh(pi x~))), and
  pi x~ = sqrt(2 pi^3 / 27) |x|^3 / (a tau0); the emergent spectrum is then
  proportional to x^2 / (1 + cosh(sqrt(2 pi^3/27) |x|^3 / (a tau0))).  The same
  route with cos((n + 1/2) pi z) modes reproduces eq. (33), which checks it.
  Normalised numerically.
* Grey symmetric birth-death chain with N interior cells: expected steps from
  cell m is m (N + 1 - m); exit probability to the right is m / (N + 1); the variance
  of the number of steps (the duration of the symmetric gambler's ruin on {0..L},
  L = N + 1, started at m) is m (L - m) (m^2 + (L - m)^2 - 2) / 3.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy import integrate

C_SLAB = math.sqrt(math.pi ** 3 / 54.0)
C_SPHERE = math.sqrt(2.0 * math.pi ** 3 / 27.0)


def neufeld_J(x, atau0):
    """Eq. (33): J(x) = x^2 / (4 sqrt(6 pi) a tau0) sech(sqrt(pi^3/54) x^3 / (a tau0))."""
    x = np.asarray(x, dtype=np.float64)
    arg = C_SLAB * x ** 3 / atau0
    return x * x / (4.0 * math.sqrt(6.0 * math.pi) * atau0) / np.cosh(np.clip(arg, -700, 700))


def slab_pdf(x, atau0):
    """Escape-frequency probability density of the slab (eq. 33 times 4 pi)."""
    return 4.0 * math.pi * neufeld_J(x, atau0)


def _sphere_shape(x, atau0):
    x = np.asarray(x, dtype=np.float64)
    arg = np.clip(C_SPHERE * np.abs(x) ** 3 / atau0, 0.0, 700.0)
    return x * x / (1.0 + np.cosh(arg))


@functools.lru_cache(maxsize=64)
def sphere_norm(atau0):
    s = (atau0 ** (1.0 / 3.0))
    val, _ = integrate.quad(lambda y: _sphere_shape(y * s, atau0), -20.0, 20.0, limit=400,
                            epsabs=0, epsrel=1e-13)
    return val * s


def sphere_pdf(x, atau0):
    return _sphere_shape(x, atau0) / sphere_norm(float(atau0))


def binned(pdf, edges, atau0):
    """Integral of ``pdf`` over each bin (probability per bin)."""
    out = np.empty(len(edges) - 1)
    for j in range(len(out)):
        out[j], _ = integrate.quad(lambda y: float(pdf(y, atau0)), edges[j], edges[j + 1],
                                   epsabs=1e-15, epsrel=1e-11, limit=200)
    return out


def slab_mode_sum(xt, n_terms=400):
    """Surface flux of the slab from its cos((n + 1/2) pi z) modes (used to check eq. 33)."""
    n = np.arange(n_terms)
    return np.sum((-1.0) ** n * np.exp(-(n + 0.5) * math.pi * abs(xt)))


def sphere_mode_sum(xt, n_terms=400):
    n = np.arange(1, n_terms + 1)
    return np.sum((-1.0) ** (n + 1) * n * np.exp(-n * math.pi * abs(xt)))


def grey_steps(N, m):
    return m * (N + 1 - m)


def grey_right_exit(N, m):
    return m / (N + 1.0)


def grey_steps_var(N, m):
    """Variance of the duration of the symmetric gambler's ruin absorbed at 0 and N + 1
    (textbook result; it vanishes for N = 1 and gives 2 for N = 2, m = 1)."""
    L = N + 1
    return m * (L - m) * (m * m + (L - m) ** 2 - 2) / 3.0
