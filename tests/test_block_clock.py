"""The cooperative walk's block clock (host-side check of its arithmetic).

The lane walk advances its FP64 clock by FP32 path lengths one step at a time.  The
cooperative walk reproduces a block of those additions as t0 + ulp * sum(rint(d / ulp)),
ulp = 2^(e-52) for t0 in [2^e, 2^(e+1)), whenever no d / ulp is exactly halfway between
integers and the result stays below 2^(e+1); otherwise it adds in order.  This checks that
premise-satisfying blocks give exactly the sequential bits, with path lengths drawn like
the walk's (-log2 of a 32-bit uniform times ln2/K, in FP32) and with values built to hit
the halfway case and the binade edge.
"""
import math

import numpy as np


def _path_lengths(rng, n, K):
    tw = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64)
    xi = ((tw.astype(np.float32) + np.float32(0.5)) * np.float32(2.3283064365386963e-10)).astype(np.float32)
    return (-np.log2(xi).astype(np.float32) * np.float32(math.log(2.0) / K)).astype(np.float32)


def _block(t0, d):
    """(parallel result or None, sequential result)."""
    seq = t0
    for v in d:
        seq = seq + float(v)
    if t0 <= 0.0:
        return None, seq
    e = math.frexp(t0)[1] - 1
    q = np.ldexp(d.astype(np.float64), 52 - e)
    if np.any(q - np.floor(q) == 0.5):
        return None, seq
    tf = t0 + math.ldexp(float(np.sum(np.rint(q))), e - 52)
    if not tf < math.ldexp(1.0, e + 1):
        return None, seq
    return tf, seq


def test_parallel_block_clock_matches_ordered_sum():
    rng = np.random.default_rng(2024)
    used = 0
    for trial in range(20000):
        t0 = float(np.exp(rng.uniform(-15, 25)))
        d = _path_lengths(rng, int(rng.integers(1, 65)), float(np.exp(rng.uniform(-8, 8))))
        par, seq = _block(t0, d)
        if par is not None:
            used += 1
            assert par == seq, (t0, d)
    assert used > 5000


def test_halfway_values_and_binade_edge_fall_back():
    # d exactly half an ulp of t0: the ordered sum's rounding depends on parity
    t0 = 1.0 + 2.0 ** -52                       # odd last bit
    d = np.array([2.0 ** -53], dtype=np.float32)
    par, seq = _block(t0, d)
    assert par is None and seq == 1.0 + 2.0 ** -51   # rounded up to the even neighbour
    assert t0 + math.ldexp(float(np.rint(0.5)), -52) == t0   # what the integer sum would give
    # a block ending exactly at (or beyond) the next power of two
    t0 = 2.0 - 2.0 ** -10
    d = np.full(4, 2.0 ** -12, dtype=np.float32)
    par, seq = _block(t0, d)
    assert par is None and seq == 2.0
    # a clock at zero adds in order
    assert _block(0.0, np.ones(3, dtype=np.float32))[0] is None
