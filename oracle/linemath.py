"""FP64 line physics -- oracle, test infrastructure only.

Follows Sec. 2.1-2.2 of the paper:
* damping parameter a(T) and thermal velocity v_th(T)             (Sec. 2.1)
* Hjerting-Voigt H(a, x), second-order expansion in a              (eq. 12)
* its integral calH(a, x) = int_0^x H(a, y) dy                      (eq. 13)
* tophat bin-averaged opacity k_j = k0 [calH(hi) - calH(lo)] / dx  (eq. 14)

erf/erfc/Dawson come from scipy.special (library routines).  Pinned in
tests/test_oracle_linemath.py against mpmath quadrature of eq. (12), against
the exact Voigt function Re w(x + i a), and against brute-force quadrature of
each bin average.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

SQRT_PI = math.sqrt(math.pi)


def damping(T):
    """a = 4.702e-4 (T / 1e4 K)^(-1/2)  (Sec. 2.1)."""
    return 4.702e-4 / np.sqrt(np.asarray(T, dtype=np.float64) / 1.0e4)


def v_thermal(T):
    """v_th = 12.85 (T / 1e4 K)^(1/2) km/s  (Sec. 2.1)."""
    return 12.85 * np.sqrt(np.asarray(T, dtype=np.float64) / 1.0e4)


def voigt_H(a, x):
    """Eq. (12): H ~= e^{-x^2} + (2a/sqrt(pi)) (2 x F(x) - 1) + a^2 e^{-x^2} (1 - 2x^2)."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-x * x)
    return e + 2.0 * a / SQRT_PI * (2.0 * x * special.dawsn(x) - 1.0) + a * a * e * (1.0 - 2.0 * x * x)


def voigt_Hcal(a, x):
    """Eq. (13): calH ~= (sqrt(pi)/2) erf(x) - (2a/sqrt(pi)) F(x) + a^2 x e^{-x^2}."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * SQRT_PI * special.erf(x) - 2.0 * a / SQRT_PI * special.dawsn(x) + a * a * x * np.exp(-x * x)


def _hcal_diff_pos(a, lo, hi):
    """calH(hi) - calH(lo) for 0 <= lo <= hi, written so that the erf difference is
    taken through erfc when both edges are in the wing (no cancellation)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    erf_part = np.where(lo > 1.0,
                        0.5 * SQRT_PI * (special.erfc(lo) - special.erfc(hi)),
                        0.5 * SQRT_PI * (special.erf(hi) - special.erf(lo)))
    daw = -2.0 * a / SQRT_PI * (special.dawsn(hi) - special.dawsn(lo))
    sq = a * a * (hi * np.exp(-hi * hi) - lo * np.exp(-lo * lo))
    return erf_part + daw + sq


def hcal_diff(a, lo, hi):
    """calH(a, hi) - calH(a, lo) for lo <= hi, any signs (calH is odd in x)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    lo, hi = np.broadcast_arrays(lo, hi)
    out = np.empty(lo.shape, dtype=np.float64)
    pos = lo >= 0.0
    neg = hi <= 0.0
    mid = ~(pos | neg)
    out[pos] = _hcal_diff_pos(a, lo[pos], hi[pos])
    out[neg] = _hcal_diff_pos(a, -hi[neg], -lo[neg])
    out[mid] = voigt_Hcal(a, hi[mid]) + voigt_Hcal(a, -lo[mid])
    return out


def bin_opacity(k0, a, lo, hi):
    """Eq. (14): tophat bin-averaged opacity over [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return k0 * hcal_diff(a, lo, hi) / (hi - lo)


def x_core_wing(a):
    """Crossover x_cw solving exp(-x^2) = a / (sqrt(pi) x^2)  (Sec. 2.1), by bisection."""
    f = lambda x: math.exp(-x * x) - a / (SQRT_PI * x * x)
    lo, hi = 1.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
