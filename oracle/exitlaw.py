"""O5: exact exit law of one DDMC cell -- oracle, test infrastructure only.

Inside cell i a DDMC packet (Sec. 2.3, eqs. 15-16) moves between the frequency bins j of the
cell with the rates of eq. (11) until a spatial leak (eq. 10, or the thin/vacuum-face rate)
takes it out through face f.  Seen from the cell, that is a finite continuous-time Markov
chain on the bins whose absorbing channels are (face, bin of the leak).  With the jump
matrix Q (tridiagonal, Q[j, j+-1] = r_j+-/K_j) and N = (I - Q)^-1:

  P(face f, bin j_out | j_in) = N[j_in, j_out] r_f(j_out) / K(j_out),
  E[steps]  = sum_j N[j_in, j],
  E[T]      = sum_j N[j_in, j] / K_j                      (c = 1),
  E[T^2]    = 2 sum_j N[j_in, j] tau_j m1_j,  m1 = N tau,  tau_j = 1 / K_j,

the same identities as the whole-medium chain (O2), restricted to one cell.  Rates come
from the oracle's own FP64 tables.  Solved with a banded LU (scipy) per entry bin.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import linalg

from . import tables as tb


@dataclasses.dataclass
class ExitLaw:
    prob: np.ndarray      # (n_faces, nb): P(face, exit bin)
    steps: float          # E[number of DDMC steps inside the cell, the leak included]
    t_mean: float         # E[time to the leak]
    t2: float             # E[time^2]

    @property
    def t_var(self):
        return self.t2 - self.t_mean ** 2


def _banded_IQ(t, cell):
    """(I - Q) of the in-cell chain in scipy's banded storage, and 1/K."""
    nb = t.nb
    dn = t.rate_dn[cell]
    up = t.rate_up[cell]
    K = t.K[cell]
    ab = np.zeros((3, nb))
    ab[1, :] = 1.0
    # row j: -Q[j, j+1] on the upper diagonal (ab[0, j+1]), -Q[j, j-1] on the lower (ab[2, j-1])
    ab[0, 1:] = -up[:-1] / K[:-1]
    ab[2, :-1] = -dn[1:] / K[1:]
    return ab, 1.0 / K


def exit_law(t, cell, j_in) -> ExitLaw:
    """Exit law of DDMC cell ``cell`` entered (or started) in bin ``j_in``; ``t`` = oracle tables."""
    nb = t.nb
    if not np.all(t.thick[cell]):
        raise ValueError("the in-cell chain needs every bin of the cell thick")
    ab, tau = _banded_IQ(t, cell)
    # v = e_jin^T N solves (I - Q)^T v = e_jin; the transpose swaps the two off-diagonals
    abT = np.zeros_like(ab)
    abT[0, 1:] = ab[2, :-1]
    abT[2, :-1] = ab[0, 1:]
    abT[1] = ab[1]
    e = np.zeros(nb)
    e[j_in] = 1.0
    v = linalg.solve_banded((1, 1), abT, e)
    m1 = linalg.solve_banded((1, 1), ab, tau)
    K = t.K[cell]
    prob = v[None, :] * t.rate_face[cell].T / K[None, :]
    return ExitLaw(prob=prob, steps=float(v.sum()), t_mean=float(v @ tau), t2=float(2.0 * np.sum(v * tau * m1)))


def exit_time_moments(t, cell, j_in):
    """E[T | exit bin j_out] and E[T^2 | exit bin j_out] for a walk entered in bin j_in, from
    first-step analysis per exit bin (columns): with h(k) = P(leak at j_out | start k),
    m(k) = E[T 1{leak at j_out} | k] and s(k) = E[T^2 1{...} | k],
      (I - Q) h = e_jout p_s(j_out),  (I - Q) m = tau h,  (I - Q) s = 2 tau m,
    (a step in k lasts tau_k on average, its square 2 tau_k^2 on average, independently of
    where it goes); then E[T | j_out] = m(j_in) / h(j_in), E[T^2 | j_out] = s(j_in) / h(j_in).
    Bins with h(j_in) = 0 get NaN."""
    nb = t.nb
    ab, tau = _banded_IQ(t, cell)
    K = t.K[cell]
    ps = t.rate_face[cell].sum(axis=1) / K
    m1 = np.full(nb, np.nan)
    m2 = np.full(nb, np.nan)
    for jo in range(nb):
        if ps[jo] <= 0.0:
            continue
        e = np.zeros(nb)
        e[jo] = ps[jo]
        h = linalg.solve_banded((1, 1), ab, e)
        m = linalg.solve_banded((1, 1), ab, tau * h)
        sq = linalg.solve_banded((1, 1), ab, 2.0 * tau * m)
        if h[j_in] > 0.0:
            m1[jo] = m[j_in] / h[j_in]
            m2[jo] = sq[j_in] / h[j_in]
    return m1, m2


def simulate(t, cell, j_in, n, seed=0, per_bin=False):
    """Brute-force sampling of the same in-cell chain (test pin for exit_law): returns
    counts (n_faces, nb), mean steps and mean time (and, with ``per_bin``, the sums of T and
    T^2 of the walks that leaked at each exit bin)."""
    rng = np.random.default_rng(seed)
    nb, nf = t.nb, t.nf
    rates = np.concatenate([t.rate_dn[cell][:, None], t.rate_up[cell][:, None], t.rate_face[cell]], axis=1)
    K = rates.sum(axis=1)
    cum = np.cumsum(rates / K[:, None], axis=1)
    counts = np.zeros((nf, nb), dtype=np.int64)
    steps = np.zeros(n)
    times = np.zeros(n)
    j = np.full(n, j_in)
    alive = np.ones(n, dtype=bool)
    t_sum = np.zeros(nb)
    t2_sum = np.zeros(nb)
    while np.any(alive):
        idx = np.nonzero(alive)[0]
        jj = j[idx]
        times[idx] += rng.exponential(1.0 / K[jj])
        steps[idx] += 1
        u = rng.random(len(idx))
        ev = (u[:, None] >= cum[jj]).sum(axis=1)        # 0 down, 1 up, 2.. faces
        ev = np.minimum(ev, 1 + nf)
        down = ev == 0
        upm = ev == 1
        j[idx[down]] -= 1
        j[idx[upm]] += 1
        leak = ev >= 2
        li = idx[leak]
        np.add.at(counts, (ev[leak] - 2, jj[leak]), 1)
        if per_bin:
            np.add.at(t_sum, jj[leak], times[li])
            np.add.at(t2_sum, jj[leak], times[li] ** 2)
        alive[li] = False
    if per_bin:
        return counts, float(steps.mean()), float(times.mean()), t_sum, t2_sum
    return counts, float(steps.mean()), float(times.mean())


def build_tables(m):
    return tb.build(m)
