"""O6: discrete frequency redistribution -- ORACLE, TEST INFRASTRUCTURE ONLY.

Sec. 5.3 (eq. 42) and Appendix A.  Plain FP64 quadrature of the printed formulas with
scipy's adaptive QUADPACK routine; nothing here is shared with the GPU library.

  r2a(x, xp, a)    Appendix A, R_II-A: the angle-averaged redistribution for isotropic
                   scattering that is coherent in the atom's frame (no recoil), in the paper's
                   normalisation -- Hummer's function divided by the incoming profile, so it is
                   the density of the outgoing x for an incoming xp: its integral over x is 1.
  r1a(x, xp)       its a -> 0 limit printed in Appendix A (pure Doppler broadening).
  r2a_wing(x, xp)  the wing limit printed in Appendix A (|x + xp| large).
  group_probability(edges, a, jp, j)
                   eq. 42 times the outgoing bin width: the probability that a packet of bin
                   jp (incoming x uniform over the bin: eq. 42 averages flatly over both bins)
                   is scattered into bin j.  Reading: the frequency grid is closed by its edge
                   bins, which take every outgoing x below the first edge (bin 0) or above the
                   last (bin nb-1), so each row sums to 1 -- the discrete analogue of the DDMC
                   grid's reflecting frequency edges.
  sample_outgoing(xp, a, rng)
                   the same law by simulation (brute force): the atom's velocity along the
                   photon from exp(-u^2) / (a^2 + (xp - u)^2), its perpendicular component
                   N(0, 1/2), an isotropic outgoing direction, and the eq. 41 frequency change
                   x = xp - u_par + u_par mu + u_perp sqrt(1 - mu^2); used to pin r2a.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate, special

_U_SPAN = 12.0     # exp(-u^2) beyond zeta + 12 is below exp(-144) of its value at zeta
_X_SPAN = 30.0     # R(x|xp) for |x - xp| > 30 is below exp(-225)


def voigt_H(a: float, x: float) -> float:
    """H(a, x) = Re w(x + i a) (Faddeeva function; H(a, 0) -> 1 as a -> 0)."""
    return float(special.wofz(complex(x, a)).real)


def r2a(x: float, xp: float, a: float, epsrel: float = 1e-11) -> float:
    """Appendix A: R_II-A(x | xp) = (1 / (pi H(a, xp))) int_zeta^inf exp(-u^2)
    [atan((x_lo + u) / a) - atan((x_hi - u) / a)] du, x_hi = max(x, xp), x_lo = min(x, xp),
    zeta = |x - xp| / 2."""
    xh, xl = max(x, xp), min(x, xp)
    zeta = 0.5 * (xh - xl)
    top = zeta + _U_SPAN

    def f(u):
        return math.exp(-u * u) * (math.atan((xl + u) / a) - math.atan((xh - u) / a))

    # the two arctangents step over a width ~a where their arguments change sign
    pts = sorted({p for p in (-xl, xh) if zeta < p < top})
    with warnings.catch_warnings():   # QUADPACK's round-off notice near 1e-11; the pins bound the error
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(f, zeta, top, points=pts or None, epsabs=0.0, epsrel=epsrel, limit=1000)
    return val / (math.pi * voigt_H(a, xp))


def r1a(x: float, xp: float) -> float:
    """Appendix A, the a -> 0 (Doppler core) form: (sqrt(pi) / 2) exp(xp^2) erfc(max(|x|, |xp|))."""
    return 0.5 * math.sqrt(math.pi) * math.exp(xp * xp) * math.erfc(max(abs(x), abs(xp)))


def r2a_wing(x: float, xp: float) -> float:
    """Appendix A, the wing form: (2 xp / (x + xp))^2 [exp(-zeta^2) / sqrt(pi) - zeta erfc(zeta)]."""
    zeta = 0.5 * abs(x - xp)
    return (2.0 * xp / (x + xp)) ** 2 * (math.exp(-zeta * zeta) / math.sqrt(math.pi) - zeta * math.erfc(zeta))


def outgoing_integral(lo: float, hi: float, xp: float, a: float, epsrel: float = 1e-11) -> float:
    """int_lo^hi R_II-A(x | xp) dx (infinite limits cut where R is below exp(-225))."""
    lo = max(lo, xp - _X_SPAN)
    hi = min(hi, xp + _X_SPAN)
    if not hi > lo:
        return 0.0
    # R has a cusp at x = xp and a step of width ~a at x = -xp
    pts = sorted({p for p in (xp, -xp) if lo < p < hi})
    val, _ = integrate.quad(lambda x: r2a(x, xp, a), lo, hi, points=pts or None, epsabs=0.0, epsrel=epsrel,
                            limit=400)
    return val


def group_probability(edges, a: float, jp: int, j: int, epsrel: float = 1e-10) -> float:
    """Eq. 42 times dx_j: P(j | jp) = (1 / dx_jp) int_{bin jp} dxp int_{bin j} R_II-A(x | xp) dx,
    with bin 0 open below and bin nb-1 open above for the outgoing x."""
    e = np.asarray(edges, dtype=np.float64)
    nb = len(e) - 1
    lo = -math.inf if j == 0 else float(e[j])
    hi = math.inf if j == nb - 1 else float(e[j + 1])
    p0, p1 = float(e[jp]), float(e[jp + 1])
    # the inner integral, as a function of xp, is not smooth where xp meets +-lo or +-hi
    pts = sorted({q for q in (lo, hi, -lo, -hi) if math.isfinite(q) and p0 < q < p1})
    val, _ = integrate.quad(lambda xp: outgoing_integral(lo, hi, xp, a, epsrel=epsrel * 0.1), p0, p1,
                            points=pts or None, epsabs=0.0, epsrel=epsrel, limit=200)
    return val / (p1 - p0)


# ---- brute force ------------------------------------------------------------------------

def _split_point(a: float, ax: np.ndarray) -> np.ndarray:
    """The split u0 in [0, |xp|] minimising the proposal mass of the sampler below (any u0 >= 0
    gives an exact sampler; this one keeps the acceptance rate high): golden-section search."""
    def mass(u0):
        th = np.arctan((u0 - ax) / a)
        return (math.pi / 2 + th) + np.exp(-u0 * u0) * (math.pi / 2 - th)
    g = 0.5 * (math.sqrt(5.0) - 1.0)
    lo, hi = np.zeros_like(ax), ax.copy()
    for _ in range(60):
        c1, c2 = hi - g * (hi - lo), lo + g * (hi - lo)
        left = mass(c1) < mass(c2)
        hi = np.where(left, c2, hi)
        lo = np.where(left, lo, c1)
    return 0.5 * (lo + hi)


def _sample_upar(xp: np.ndarray, a: float, rng: np.random.Generator) -> np.ndarray:
    """Atom velocity along the photon, density ~ exp(-u^2) / (a^2 + (xp - u)^2), by rejection
    from a Lorentzian split at u0 >= 0 (the method of Zheng & Miralda-Escude 2002), on |xp| and
    mirrored: below u0 the proposal is the Lorentzian 1 / (a^2 + (|xp| - u)^2), accepted with
    probability exp(-u^2) <= 1; above u0 it is exp(-u0^2) times the Lorentzian, accepted with
    probability exp(u0^2 - u^2) <= 1."""
    ax = np.abs(np.asarray(xp, dtype=np.float64))
    u0 = _split_point(a, ax)
    th0 = np.arctan((u0 - ax) / a)
    e0 = np.exp(-u0 * u0)
    m1 = th0 + math.pi / 2                      # Lorentzian mass below u0 (times a)
    m2 = e0 * (math.pi / 2 - th0)               # exp(-u0^2) times the mass above u0
    out = np.empty_like(ax)
    todo = np.arange(ax.size)
    while todo.size:
        k = todo.size
        low = rng.random(k) * (m1[todo] + m2[todo]) < m1[todo]
        th = np.where(low, -math.pi / 2 + m1[todo] * rng.random(k),
                      th0[todo] + (math.pi / 2 - th0[todo]) * rng.random(k))
        u = ax[todo] + a * np.tan(th)
        acc = np.where(low, np.exp(-u * u), np.exp(u0[todo] ** 2 - u * u))
        ok = rng.random(k) < acc
        out[todo[ok]] = u[ok]
        todo = todo[~ok]
    return np.where(np.asarray(xp) < 0, -out, out)


def sample_outgoing(xp: np.ndarray, a: float, rng: np.random.Generator) -> np.ndarray:
    """Outgoing comoving x of one isotropic scattering, coherent in the atom frame (eq. 41
    without recoil), for each incoming xp."""
    xp = np.asarray(xp, dtype=np.float64)
    upar = _sample_upar(xp, a, rng)
    uperp = rng.standard_normal(xp.shape) / math.sqrt(2.0)
    mu = 2.0 * rng.random(xp.shape) - 1.0
    return xp + upar * (mu - 1.0) + uperp * np.sqrt(1.0 - mu * mu)


def sample_group(edges, a: float, jp: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """Outgoing bins of n packets of bin jp (incoming x uniform in the bin), edge bins open."""
    e = np.asarray(edges, dtype=np.float64)
    xp = e[jp] + (e[jp + 1] - e[jp]) * rng.random(n)
    x = sample_outgoing(xp, a, rng)
    return np.clip(np.searchsorted(e, x, side="right") - 1, 0, len(e) - 2)
