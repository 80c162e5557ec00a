"""O2: exact pure-DDMC chain -- oracle, test infrastructure only.

In pure DDMC every state (cell, bin) is a state of a finite continuous-time
Markov chain whose rates are the leakage coefficients of eqs. (10) and (11)
(Sec. 2.2); the walk of Sec. 2.3 (eqs. 15-16: the smallest of independent
exponential distances) samples its absorption at the domain boundary.  So the
expected escape spectrum, the expected number of leakage events and the
moments of the escape time are solutions of sparse linear systems:

  P = rates / K (jump matrix),  v = (I - P)^-T pi0  (expected visits),
  p(face, bin) = sum_s v_s r_esc(s -> face, bin) / K_s,
  E[steps] = sum_s v_s,  E[T] = sum_s v_s / K_s  (c = 1),
  (I - P) m1 = tau, E[T^2] = 2 sum_s v_s tau_s m1_s, with tau_s = 1 / K_s.

Dust (Sec. 2.4): the leakage coefficients use the total scattering coefficient (the tables add
the dust scattering k_s), and absorption is one more exponential channel of rate k_a, so
K_s = sum of leakage rates + k_a and the chain is absorbed with probability
sum_s v_s k_a / K_s.  Escape-time moments are then conditioned on escape: with h the
escape probability from each state ((I - P) h = the one-step escape probability),
(I - P) u = tau h gives E[T 1_esc] = v . (tau h) and E[T^2 1_esc] = 2 v . (tau u).

The transient law (time-dependent estimators of eq. 17): the occupation probabilities
p(t) = p0 exp(Q t) of the generator Q = rates - diag(K), at census times and averaged over
the intervals between them; with an emission window [t_s, t_e] the law is the flash law
averaged over emission times.

With bulk velocity a spatial move draws x uniformly in the bin, maps it to the
neighbour's frame (Sec. 2.5) and re-bins it; the exact transition weights are
the overlaps of the shifted bin with the neighbour's bins (parts outside the
grid go to the edge bins).  An escaping packet's lab-frame frequency is x + n.u with x
uniform in its bin and n an isotropic outward direction (mu uniform in (0, 1]); in 1D
geometries the velocity is normal to the faces and this is x + mu u_n.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import tables as tb


@dataclasses.dataclass
class ChainResult:
    spectrum: np.ndarray      # (n_escape_faces, nb + 2) escape probability per face and lab bin
    faces: list               # face ids of the rows of spectrum
    steps: float              # E[number of leakage events] (an absorption counts as one)
    steps2: float             # E[steps^2]
    t_mean: float             # E[escape time | escaped] (length / c)
    t2: float                 # E[escape time^2 | escaped]
    visits: np.ndarray        # expected visits per state (nc, nb)
    total: float              # sum of all escape probabilities (1 without dust)
    absorbed: float = 0.0     # probability of absorption by dust (Sec. 2.4)

    @property
    def t_var(self):
        return self.t2 - self.t_mean ** 2

    @property
    def steps_var(self):
        return self.steps2 - self.steps ** 2

    def spectrum_total(self):
        return self.spectrum.sum(axis=0)


def _overlap_matrix(edges, lo, hi):
    """Fraction of [lo, hi] falling in each bin of ``edges``; the parts below/above the
    grid are added to the first/last bin.  Returns (bin indices, weights)."""
    nb = len(edges) - 1
    w = hi - lo
    jlo = max(0, int(np.searchsorted(edges, lo, side="right")) - 1)
    jhi = min(nb - 1, int(np.searchsorted(edges, hi, side="left")) - 1)
    jlo = min(jlo, nb - 1)
    jhi = max(jhi, 0)
    idx, wt = [], []
    for j in range(jlo, jhi + 1):
        a = max(lo, edges[j]) if j > 0 else lo
        b = min(hi, edges[j + 1]) if j < nb - 1 else hi
        if b > a:
            idx.append(j)
            wt.append((b - a) / w)
    if not idx:   # degenerate: entirely outside the grid
        idx = [0 if hi <= edges[0] else nb - 1]
        wt = [1.0]
    wt = np.asarray(wt)
    return np.asarray(idx), wt / wt.sum()


def _overlaps(edges, A, B):
    """All bins' images [A_j, B_j] re-binned on ``edges``: returns (j, j', weight) triples
    with weight = fraction of [A_j, B_j] inside bin j' (parts below / above the grid are
    given to the first / last bin).  Same rule as _overlap_matrix, vectorised over j."""
    nb = len(edges) - 1
    w = B - A
    first = np.clip(np.searchsorted(edges, A, side="right") - 1, 0, nb - 1)
    last = np.clip(np.searchsorted(edges, B, side="left") - 1, 0, nb - 1)
    span = int((last - first).max()) + 1
    js, jd, wt = [], [], []
    for d in range(span):
        jp = first + d
        ok = jp <= last
        lo = np.where(jp > 0, np.maximum(A, edges[np.minimum(jp, nb)]), A)
        hi = np.where(jp < nb - 1, np.minimum(B, edges[np.minimum(jp + 1, nb)]), B)
        frac = np.clip(hi - lo, 0.0, None) / w
        ok &= frac > 0
        js.append(np.nonzero(ok)[0])
        jd.append(jp[ok])
        wt.append(frac[ok])
    js, jd, wt = np.concatenate(js), np.concatenate(jd), np.concatenate(wt)
    tot = np.bincount(js, weights=wt, minlength=len(A))
    return js, jd, wt / tot[js]


def _ramp_area(t):
    t = np.maximum(t, 0.0)
    return 0.5 * t * t


def lab_bin_probs(edges, lo, hi, u):
    """P(x + mu u in lab bin b) for x ~ U[lo, hi], mu ~ U(0, 1]; b over the nb+2 lab
    slots (0 = below the grid, nb+1 = above)."""
    nb = len(edges) - 1
    out = np.zeros(nb + 2)
    if abs(u) < 1e-300:
        cdf = np.clip((edges - lo) / (hi - lo), 0.0, 1.0)
    else:
        a2, b2 = (0.0, u) if u > 0 else (u, 0.0)
        area = (hi - lo) * (b2 - a2)
        y = edges
        cdf = (_ramp_area(y - lo - a2) - _ramp_area(y - hi - a2) - _ramp_area(y - lo - b2)
               + _ramp_area(y - hi - b2)) / area
        cdf = np.where(y >= hi + b2, 1.0, np.where(y <= lo + a2, 0.0, np.clip(cdf, 0.0, 1.0)))
        cdf = np.maximum.accumulate(cdf)
    out[0] = cdf[0]
    out[1:nb + 1] = np.diff(cdf)
    out[nb + 1] = 1.0 - cdf[-1]
    return out


def lab_bin_probs_3d(edges, lo, hi, u_n, u_t, n_mu=64, n_phi=64):
    """P(x + n.u in lab bin b) for x ~ U[lo, hi] and an isotropic outward direction n
    (mu = n.n_face uniform in (0, 1], azimuth uniform): the shift is
    mu u_n + sqrt(1 - mu^2) u_t cos(phi).  Gauss-Legendre in mu, trapezoid (periodic,
    spectrally accurate) in phi."""
    if u_t == 0.0:
        return lab_bin_probs(edges, lo, hi, u_n)
    nb = len(edges) - 1
    gx, gw = np.polynomial.legendre.leggauss(n_mu)
    mu = 0.5 * (gx + 1.0)
    wmu = 0.5 * gw
    phi = 2.0 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    shift = (mu[:, None] * u_n + np.sqrt(1.0 - mu[:, None] ** 2) * u_t * np.cos(phi[None, :])).ravel()
    wts = (wmu[:, None] * np.full(n_phi, 1.0 / n_phi)[None, :]).ravel()
    a = lo + shift
    b = hi + shift
    y = np.asarray(edges)
    cdf = np.clip((y[None, :] - a[:, None]) / (b - a)[:, None], 0.0, 1.0)   # (nodes, nb+1)
    # per-node slot masses (each >= 0, exactly 0 outside the node's support), then the
    # weighted mean: no cancellation between cumulative sums
    slots = np.concatenate([cdf[:, :1], np.diff(cdf, axis=1), 1.0 - cdf[:, -1:]], axis=1)
    return (wts @ slots) / wts.sum()


def _chain(m, tabs=None):
    """The sparse chain of pure DDMC on medium ``m``: transient-to-transient rates, total
    rates K (leakage plus dust absorption), escape channels and the emission law."""
    t = tabs if tabs is not None else tb.build(m)
    if not np.all(t.thick):
        raise ValueError("the exact chain covers pure DDMC only (every state thick)")
    nc, nb, nf = t.nc, t.nb, t.nf
    ns = nc * nb
    k_abs = np.zeros(nc) if t.k_abs is None else t.k_abs
    K = (t.K + k_abs[:, None]).reshape(ns)
    edges = t.bin_edges
    rows, cols, vals = [], [], []
    sidx = np.arange(ns).reshape(nc, nb)
    # frequency moves
    for dj, r in ((-1, t.rate_dn), (1, t.rate_up)):
        mask = r > 0
        s_from = sidx[mask]
        s_to = s_from + dj
        rows.append(s_from)
        cols.append(s_to)
        vals.append(r[mask])
    esc_faces = sorted({f for f in range(nf) if np.any(t.nbr[:, f] == tb.NBR_VACUUM)})
    face_row = {f: i for i, f in enumerate(esc_faces)}
    es, ef, eb, er = [], [], [], []   # escape channels: (state, face row, lab slot, rate)
    lo_e, hi_e = edges[:-1], edges[1:]
    for f in range(nf):
        static_f = (t.rho[:, f] == 1.0) & (t.shift[:, f] == 0.0) & (t.nbr[:, f] >= 0)
        if np.any(static_f):
            cs = np.nonzero(static_f)[0]
            r = t.rate_face[cs, :, f]
            mask = r > 0
            src_s = (cs[:, None] * nb + np.arange(nb)[None, :])[mask]
            dst_s = (t.nbr[cs, f][:, None] * nb + np.arange(nb)[None, :])[mask]
            rows.append(src_s)
            cols.append(dst_s)
            vals.append(r[mask])
        vac_static = (t.nbr[:, f] == tb.NBR_VACUUM) & (((t.u_n[:, f] == 0.0) & (t.u_t[:, f] == 0.0))
                                                       | (not t.moving))
        if np.any(vac_static):
            cs = np.nonzero(vac_static)[0]
            jj = np.arange(nb)
            es.append((cs[:, None] * nb + jj[None, :]).ravel())
            ef.append(np.full(len(cs) * nb, face_row[f]))
            eb.append(np.tile(jj + 1, len(cs)))
            er.append(t.rate_face[cs, :, f].ravel())
        for c in range(nc):
            n = t.nbr[c, f]
            r = t.rate_face[c, :, f]
            if n == tb.NBR_NONE or static_f[c] or vac_static[c]:
                continue
            if n == tb.NBR_VACUUM:
                u = t.u_n[c, f] if t.moving else 0.0
                ut = t.u_t[c, f] if t.moving else 0.0
                for j in range(nb):
                    if r[j] <= 0:
                        continue
                    pb = lab_bin_probs_3d(edges, lo_e[j], hi_e[j], u, ut)
                    nzb = np.nonzero(pb)[0]
                    es.append(np.full(len(nzb), c * nb + j))
                    ef.append(np.full(len(nzb), face_row[f]))
                    eb.append(nzb)
                    er.append(r[j] * pb[nzb])
                continue
            rho, sh = t.rho[c, f], t.shift[c, f]
            src_j, dst_j, wts = _overlaps(edges, rho * lo_e + sh, rho * hi_e + sh)
            keep = r[src_j] > 0
            rows.append(c * nb + src_j[keep])
            cols.append(n * nb + dst_j[keep])
            vals.append(r[src_j[keep]] * wts[keep])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    R = sp.csr_matrix((np.concatenate(vals), (rows, cols)), shape=(ns, ns))
    pi0 = np.zeros(ns)
    for st, pr in tb.locate_sources(m):
        pi0[st] += pr
    es, ef, eb, er = (np.concatenate(z) for z in (es, ef, eb, er))
    return dict(t=t, ns=ns, nb=nb, K=K, R=R, pi0=pi0, esc=(es, ef, eb, er), faces=esc_faces,
                k_abs=np.repeat(k_abs, nb))


def solve(m, tabs=None) -> ChainResult:
    """Exact expected results of pure DDMC on medium ``m``."""
    ch = _chain(m, tabs)
    ns, nb, K, R, pi0 = ch["ns"], ch["nb"], ch["K"], ch["R"], ch["pi0"]
    es, ef, eb, er = ch["esc"]
    nc = ns // nb
    P = sp.diags(1.0 / K) @ R
    A = (sp.identity(ns, format="csr") - P).tocsc()
    lu = spla.splu(A)
    v = lu.solve(pi0, trans="T")
    tau = 1.0 / K
    n1 = lu.solve(np.ones(ns))
    nrow = len(ch["faces"])
    spec = np.bincount(ef * (nb + 2) + eb, weights=(v / K)[es] * er,
                       minlength=nrow * (nb + 2)).reshape(nrow, nb + 2)
    # escape probability from each state (1 without dust)
    esc1 = np.bincount(es, weights=er, minlength=ns) / K
    h = lu.solve(esc1)
    u = lu.solve(tau * h)
    p_esc = float(pi0 @ h)
    steps = float(v.sum())
    steps2 = float(v @ (2.0 * n1 - 1.0))
    t_mean = float(v @ (tau * h)) / p_esc
    t2 = float(2.0 * v @ (tau * u)) / p_esc
    absorbed = float(v @ (ch["k_abs"] / K))
    return ChainResult(spectrum=spec, faces=ch["faces"], steps=steps, steps2=steps2, t_mean=t_mean,
                       t2=t2, visits=v.reshape(nc, nb), total=float(spec.sum()), absorbed=absorbed)


@dataclasses.dataclass
class TransientResult:
    edges: np.ndarray         # census times t_0 < ... < t_n
    at_edges: np.ndarray      # (n+1, nc, nb): P(the packet is in state s at t_e)
    mean_in: np.ndarray       # (n, nc, nb): the occupation averaged over [t_e, t_e+1)
    escaped_by: np.ndarray    # (n+1,): P(escaped by t_e)
    accel: np.ndarray = None  # (n, nc): eq. 18's optical-depth sum per cell and interval (1D)


def _accel_weights(ch, dust_weights=False):
    """Per state s = (c, j): the expected eq. 18 contribution of one unit of residence in s,
    split into the cell it leaks out of and the cell it leaks into.  A step in s lasts
    dl ~ Exp(K_s) and ends in leak f with probability r_f / K_s, independently of dl; a leak
    along direction d (-1 through face 0, +1 through face 1) adds k_s dl d to cell c and, when
    the neighbour c' is a grid cell, k_{c',j'} dl d to c' at the bin j' it lands in (Doppler
    re-binning of eq. 20 for moving media).  Returns (out (ns,), into list of (dst cell,
    weights (ns,))).

    With ``dust_weights`` (Sec. 2.4's continuous weights) absorption is not an event: a step
    lasts dl ~ Exp(K_leak) and ends in leak f with probability r_f / K_leak, and the leak adds
    k d times the weight integrated over the step (the paper's path correction); the expected
    weighted residence in s is the killed chain's, so the weights per unit residence are
    r_f / K_leak instead of r_f / (K_leak + k_a)."""
    t, nb, K = ch["t"], ch["nb"], ch["K"]
    nc = t.nc
    if t.nf != 2:
        raise ValueError("the acceleration estimator is tallied on 1D grids (slab z, sphere r)")
    kk = t.k
    edges = t.bin_edges
    out = np.zeros(nc * nb)
    into = np.zeros((nc, nc * nb))
    Kstep = t.K if dust_weights else K.reshape(nc, nb)       # the rate that ends a step
    for f, d in ((0, -1.0), (1, 1.0)):
        p = t.rate_face[:, :, f] / Kstep                      # P(leak through f | s)
        out += (d * p * kk).ravel()
        for c in range(nc):
            n = t.nbr[c, f]
            if n < 0:
                continue
            rho, sh = t.rho[c, f], t.shift[c, f]
            if rho == 1.0 and sh == 0.0:
                kn = kk[n]
            else:
                src_j, dst_j, wts = _overlaps(edges, rho * edges[:-1] + sh, rho * edges[1:] + sh)
                kn = np.bincount(src_j, weights=wts * kk[n][dst_j], minlength=nb)
            into[n, c * nb:(c + 1) * nb] += d * p[c] * kn
    return out, into


def transient(m, edges, tabs=None, emit=None, dust_weights=False) -> TransientResult:
    """Transient law of pure DDMC on a small medium (dense matrices): the expectations, per
    emitted packet, of the 'bin' estimator at each census time and of the 'path' estimator
    over each census interval (eq. 17, without the energy and volume factors).  ``emit`` =
    (t_s, t_e) emits packets uniformly in time over that window (t_e > t_s), else a flash at
    t = 0.  ``dust_weights``: eq. 18's expectation under continuous dust weights (see
    _accel_weights); the occupation and residence expectations are the same for both dust
    methods."""
    from scipy import linalg as la
    ch = _chain(m, tabs)
    ns, nb, K, R, pi0 = ch["ns"], ch["nb"], ch["K"], ch["R"], ch["pi0"]
    if ns > 4000:
        raise ValueError("the dense transient solve is for small media")
    es, ef, eb, er = ch["esc"]
    Q = R.toarray() - np.diag(K)
    esc_rate = np.bincount(es, weights=er, minlength=ns)
    Qi = la.inv(Q)
    edges = np.asarray(edges, dtype=np.float64)

    def E(t):     # exp(Q t), t >= 0
        return la.expm(Q * t)

    def F(t):     # int_0^t exp(Q s) ds
        return Qi @ (E(t) - np.eye(ns)) if t > 0 else np.zeros((ns, ns))

    def G(t):     # int_0^t F(s) ds
        return Qi @ (F(t) - t * np.eye(ns)) if t > 0 else np.zeros((ns, ns))

    def occ(t):   # P(in state s at time t)
        if emit is None:
            return pi0 @ E(t)
        ts, te = emit
        return pi0 @ (F(max(t - ts, 0.0)) - F(max(t - te, 0.0))) / (te - ts)

    def occ_int(t):   # int_0^t occ
        if emit is None:
            return pi0 @ F(t)
        ts, te = emit
        return pi0 @ (G(max(t - ts, 0.0)) - G(max(t - te, 0.0))) / (te - ts)

    at = np.array([occ(t) for t in edges])
    cum = np.array([occ_int(t) for t in edges])
    mean = (cum[1:] - cum[:-1]) / np.diff(edges)[:, None]
    # escaped by t: the escape flux integrated, int_0^t occ . esc_rate
    escaped = cum @ esc_rate
    nc = ns // nb
    accel = None
    if ch["t"].nf == 2:
        res = cum[1:] - cum[:-1]                    # expected residence per (interval, state)
        w_out, w_into = _accel_weights(ch, dust_weights)
        accel = (res * w_out).reshape(len(edges) - 1, nc, nb).sum(axis=2) + res @ w_into.T
    return TransientResult(edges=edges, at_edges=at.reshape(len(edges), nc, nb),
                           mean_in=mean.reshape(len(edges) - 1, nc, nb), escaped_by=escaped, accel=accel)
