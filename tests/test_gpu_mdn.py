"""GPU mixture-density network (BF16 MFMA, FP32 accumulation) against the FP64 oracle O4:
outputs, loss and the backpropagated gradient at the same parameters; training lowers
the loss of a known law."""
import math

import numpy as np
import pytest

from oracle import mdn as omdn
from paper_1709_10187_amd import rddmc

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, omdn.D_IN))
    X[:, :8] = rng.normal(size=(n, 8))
    Y = np.stack([rng.integers(0, 2, size=n), rng.normal(size=n), rng.normal(1.0, 0.5, size=n)], axis=1)
    return X, Y


def _theta(seed=3):
    th = omdn.init(seed) * 1.3
    th += np.random.default_rng(seed).normal(scale=0.02, size=th.shape)
    return th.astype(np.float32).astype(np.float64)     # the GPU holds FP32 parameters


@pytest.mark.parametrize("n", [64, 200, 4096])
def test_forward_and_gradient_match_fp64_oracle(n):
    import torch
    print(f"[mdn] forward/gradient vs FP64 oracle, batch {n}", flush=True)
    th = _theta()
    X, Y = _batch(n, 5)
    net = rddmc.Mdn(max_batch=4096)
    net.set_theta(th)
    x = torch.tensor(X, dtype=torch.float32, device="cuda")
    y = torch.tensor(Y, dtype=torch.float32, device="cuda")
    out = net.forward(x).cpu().numpy().astype(np.float64)
    ref = omdn.forward(th, X.astype(np.float32).astype(np.float64))
    # BF16 operands (8-bit mantissa) through four layers
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    assert err < 2e-2, err
    loss = float(net.loss_grad(x, y).cpu()[0])
    ref_loss, ref_g = omdn.loss_and_grad(th, X.astype(np.float32).astype(np.float64), Y)
    assert loss == pytest.approx(ref_loss, rel=2e-2)
    _, g = net.get()
    g = g.astype(np.float64)
    rel = np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g)
    cos = float(g @ ref_g / (np.linalg.norm(g) * np.linalg.norm(ref_g)))
    print(f"    out rel err {err:.2e}  loss {loss:.5f} vs {ref_loss:.5f}  grad rel err {rel:.2e}  cos {cos:.6f}",
          flush=True)
    assert rel < 2e-2 and cos > 0.999
    # per layer block as well (no block may hide behind the others)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in omdn.SHAPES])
    for b in range(len(omdn.SHAPES)):
        gb, rb = g[offs[b]:offs[b + 1]], ref_g[offs[b]:offs[b + 1]]
        if np.linalg.norm(rb) > 0:
            assert np.linalg.norm(gb - rb) / np.linalg.norm(rb) < 5e-2, b


def test_training_lowers_the_loss_of_a_known_law():
    """Targets drawn from a law that depends on the inputs: face = [x0 > 0], y1 ~ N(x1, 0.1),
    y2 ~ N(0.5 x2, 0.2).  Adam on the GPU brings the NLL near the law's own entropy."""
    import torch
    rng = np.random.default_rng(9)
    n = 4096
    net = rddmc.Mdn(max_batch=n, seed=1)
    first = last = None
    for it in range(300):
        X = np.zeros((n, omdn.D_IN))
        X[:, :3] = rng.normal(size=(n, 3))
        Y = np.stack([(X[:, 0] > 0).astype(float), rng.normal(X[:, 1], 0.1), rng.normal(0.5 * X[:, 2], 0.2)], axis=1)
        x = torch.tensor(X, dtype=torch.float32, device="cuda")
        y = torch.tensor(Y, dtype=torch.float32, device="cuda")
        loss = float(net.train_step(x, y, 2e-3).cpu()[0])
        if it == 0:
            first = loss
        last = loss
    # entropy of the law: 0 (face) + 0.5 log(2 pi e 0.1^2) + 0.5 log(2 pi e 0.2^2)
    h = 0.5 * math.log(2 * math.pi * math.e * 0.01) + 0.5 * math.log(2 * math.pi * math.e * 0.04)
    print(f"[mdn] training: loss {first:.3f} -> {last:.3f} (law entropy {h:.3f})", flush=True)
    assert last < first - 2.0
    assert last < h + 0.5
