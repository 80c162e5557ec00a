"""The weighted-spectrum statistics used by the dust-weight tests: with unit weights they are
the binomial statistics of plain counts, and they flag a shifted sample."""
import numpy as np

from tests._stats import compare_exact, compare_weighted_exact, compare_weighted_two


def test_unit_weights_reduce_to_counts():
    rng = np.random.default_rng(5)
    p = rng.dirichlet(np.ones(40))
    n = 200_000
    counts = rng.multinomial(n, p).astype(np.float64)
    rw = compare_weighted_exact(counts, counts, n, p)
    rc = compare_exact(counts, p, n)
    np.testing.assert_allclose(rw["z"], rc["z"], rtol=0.05, atol=0.05)
    assert rw["p_value"] > 1e-3


def test_weighted_two_samples_detect_a_shift():
    rng = np.random.default_rng(6)
    p = rng.dirichlet(np.ones(30))
    n = 100_000
    a = rng.multinomial(n, p).astype(np.float64)
    b = rng.multinomial(n, p).astype(np.float64)
    same = compare_weighted_two(a, a, n, b, b, n)
    assert same["p_value"] > 1e-3
    q = np.roll(p, 1)
    c = rng.multinomial(n, q).astype(np.float64)
    diff = compare_weighted_two(a, a, n, c, c, n)
    assert diff["p_value"] < 1e-6
