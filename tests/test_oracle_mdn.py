"""Pins of the FP64 mixture-density network (O4): the likelihood against scipy's bivariate
normal and log-sum-exp, the output gradient and the full backpropagated gradient against
central finite differences."""
import math

import numpy as np
import pytest
from scipy import special, stats

from oracle import mdn


def _random_batch(n=6, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, mdn.D_IN))
    X[:, 8:] = 0.0
    Y = np.stack([rng.integers(0, 2, size=n), rng.normal(size=n), rng.normal(1.0, 0.5, size=n)], axis=1)
    return X, Y


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mdn.gelu(z), z * stats.norm.cdf(z), rtol=1e-12, atol=1e-300)
    h = 1e-6
    np.testing.assert_allclose(mdn.gelu_grad(z), (mdn.gelu(z + h) - mdn.gelu(z - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_nll_against_scipy_bivariate_normal():
    rng = np.random.default_rng(3)
    n = 5
    o = rng.normal(scale=0.7, size=(n, mdn.D_OUT))
    _, Y = _random_batch(n, 4)
    got = mdn.nll(o, Y)
    a, fl, mu1, s1, mu2, s2, rho = mdn.split(o)
    for i in range(n):
        f = int(Y[i, 0])
        terms = []
        for k in range(mdn.N_COMP):
            pi = special.softmax(a[i])[k]
            pf = special.softmax(fl[i, k])[f]
            sg1, sg2, r = math.exp(s1[i, k]), math.exp(s2[i, k]), rho[i, k]
            cov = [[sg1 * sg1, r * sg1 * sg2], [r * sg1 * sg2, sg2 * sg2]]
            terms.append(pi * pf * stats.multivariate_normal(mean=[mu1[i, k], mu2[i, k]], cov=cov).pdf(Y[i, 1:]))
        assert got[i] == pytest.approx(-math.log(sum(terms)), rel=1e-10)


def test_output_gradient_finite_differences():
    rng = np.random.default_rng(5)
    n = 4
    o = rng.normal(scale=0.8, size=(n, mdn.D_OUT))
    _, Y = _random_batch(n, 6)
    g = mdn.nll_grad_out(o, Y)
    h = 1e-6
    # central differences carry ~eps |loss| / h ~ 2e-9 of rounding: the absolute floor
    floor = 20 * np.finfo(float).eps * abs(mdn.nll(o, Y).mean()) / h
    for i in range(n):
        for j in range(mdn.D_OUT):
            op, om = o.copy(), o.copy()
            op[i, j] += h
            om[i, j] -= h
            fd = (mdn.nll(op, Y).mean() - mdn.nll(om, Y).mean()) / (2 * h)
            assert g[i, j] == pytest.approx(fd, rel=1e-6, abs=floor), (i, j)


def test_parameter_gradient_finite_differences():
    theta = mdn.init(seed=1) * 1.5
    rng = np.random.default_rng(7)
    theta += rng.normal(scale=0.02, size=theta.shape)   # non-zero biases too
    X, Y = _random_batch(8, 8)
    loss, g = mdn.loss_and_grad(theta, X, Y)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in mdn.SHAPES])
    h = 1e-6
    floor = 20 * np.finfo(float).eps * abs(loss) / h     # rounding of the central difference
    worst = 0.0
    for b in range(len(mdn.SHAPES)):
        for idx in rng.integers(offs[b], offs[b + 1], size=6):
            tp, tm = theta.copy(), theta.copy()
            tp[idx] += h
            tm[idx] -= h
            fd = (mdn.nll(mdn.forward(tp, X), Y).mean() - mdn.nll(mdn.forward(tm, X), Y).mean()) / (2 * h)
            err = abs(g[idx] - fd) / (1e-6 * abs(fd) + floor)
            worst = max(worst, err)
    assert worst < 1.0
    assert loss == pytest.approx(float(mdn.nll(mdn.forward(theta, X), Y).mean()), rel=1e-14)
