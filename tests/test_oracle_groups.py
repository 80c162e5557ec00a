"""Pins of the oracle walker's frequency-group mode (Sec. 5.3): in an optically thin slab a
packet escapes unscattered with the probability E_2(tau) of a central isotropic source, and
the packets that scatter once leave with the bins of eq. 42 (O6, independent of the walker);
second scatterings are of relative order tau ln(1/tau).  Checked bin by bin within 4 standard
deviations."""
import numpy as np
from scipy import special

from oracle import redistribution as rd
from oracle import tables as tb
from oracle import walk1dh
from paper_1709_10187_amd import media

EDGES = np.array([-8.0, -5.0, -3.2, -1.0, 1.0, 3.2, 5.0, 8.0])


def thin_group_slab(tau_src, n_packets, n_cells=4):
    """Static slab z in [-1, 1], T = 1e4 K, every state thin, source at z = 0 in bin 3
    (x = 0), k0 set so that the source bin's averaged opacity times the half-width is tau_src."""
    m = media.slab(1.0, 1e4, n_cells, len(EDGES) - 1).replace(
        bin_edges=EDGES, tau_threshold=media.ALL_THIN, flags=media.GROUP_MC, n_packets=int(n_packets))
    k_src = tb.build(m).k[0, 3]
    return m.replace(k0=np.full(n_cells, tau_src / k_src))


def test_single_scattering_limit():
    tau, n = 1e-4, 40_000_000
    m = thin_group_slab(tau, n)
    res = walk1dh.run(m, seed=3)
    assert res.escaped == n and res.to_ddmc == 0
    spec = res.spectrum.sum(axis=0)[1:-1].astype(np.float64)
    p_sc = 1.0 - special.expn(2, tau)
    row = np.array([rd.group_probability(EDGES, media._a_of_T(1e4), 3, j, epsrel=1e-6) for j in range(7)])
    want = n * p_sc * row
    want[3] += n * (1.0 - p_sc)
    var = n * p_sc * row * (1.0 - p_sc * row)        # the scattered part carries the noise
    z = (spec - want) / np.sqrt(np.maximum(var, 1.0))
    assert np.all(np.abs(z) < 4.0), (spec, want, z)
    assert want[2] > 1500 and want[4] > 1500          # the test has power in the wings
