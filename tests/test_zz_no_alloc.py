"""rddmc_transport_static (the allocation-free entry point) against rddmc_transport: the same
walk with the library's own device work area gives the same integer tallies, bit for bit, on
two calls in a row (the second with a smaller input), for a 1D cloud whose tail goes through
the cooperative walk and for a 3D hybrid cube."""
import numpy as np
import pytest
import torch

from paper_1709_10187_amd import media, rddmc

pytestmark = pytest.mark.gpu


def _words(prob):
    return prob.tallies.cpu().numpy().copy()


def _pair(m, **kw):
    print(f"no-alloc: {m.name} {kw}", flush=True)
    ref = rddmc.Problem(m)
    ref.run(**kw)
    got = rddmc.Problem(m)
    rddmc.transport_static(got.batch, got.tables, got.tallies, **kw)
    torch.cuda.synchronize()
    a, b = _words(ref), _words(got)
    res = got.results()[0]
    return a, b, res


@pytest.mark.parametrize("kind", ["slab", "cube"])
def test_static_work_area_matches_transport(kind):
    torch.cuda.set_device(0)
    if kind == "slab":
        big = media.slab(3.0e3, 1.0e4, 16, 32, n_packets=40000,
                         vel=np.linspace(-30.0, 30.0, 16), name="slab_moving")
        small = media.slab(1.0e3, 1.0e4, 8, 16, n_packets=3000, name="slab_small")
        runs = [(big, dict(seed=5, tail_lanes=32)), (small, dict(seed=6, block=128, grid=7, chunk=9))]
    else:
        big = media.cube(n=12, n_bins=48, n_sources=8, packets_per_source=4096, name="cube12")
        small = media.cube(n=6, n_bins=32, n_sources=4, packets_per_source=512, name="cube6")
        runs = [(big, dict(seed=3)), (small, dict(seed=4, block=64, grid=9))]
    for m, kw in runs:          # two calls in a row, the second smaller
        a, b, res = _pair(m, **kw)
        assert res.launched == m.n_packets and res.escaped + res.capped == m.n_packets
        np.testing.assert_array_equal(a, b)


def test_static_rejects_grids_beyond_the_work_area():
    m = media.slab(1.0e3, 1.0e4, 8, 16, n_packets=1000)
    p = rddmc.Problem(m)
    with pytest.raises(rddmc.RddmcError) as ei:
        rddmc.transport_static(p.batch, p.tables, p.tallies, block=256, grid=(1 << 19) // 256 + 1)
    assert ei.value.status == -2
    rddmc.transport_static(p.batch, p.tables, p.tallies, block=256, grid=(1 << 19) // 256)
    torch.cuda.synchronize()
    assert p.results()[0].escaped == 1000
