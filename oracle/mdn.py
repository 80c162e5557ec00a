"""O4: FP64 mixture-density network -- oracle, test infrastructure only.

The learned escape surrogate maps the description of one thick DDMC cell and the packet's
entry bin to the law of its exit from the cell: face, exit frequency and time spent.  The
network is a plain multilayer perceptron,

  h1 = gelu(x W1 + b1),  h2 = gelu(h1 W2 + b2),  h3 = gelu(h2 W3 + b3),  o = h3 W4 + b4,

with exact (erf) GELU, widths 16 -> 256 -> 256 -> 256 -> 128.  The 128 outputs are a
16-component mixture; component k has
  o[k]                 mixture logit,
  o[16 + 2k + f]       logit of exit face f (f = 0, 1),
  o[48 + k], o[64 + k] mean and log-sigma of y1 (asinh-scaled exit frequency),
  o[80 + k], o[96 + k] mean and log-sigma of y2 (log time),
  o[112 + k]           correlation raw value, rho = 0.95 tanh(.),
with log-sigma clamped to [-6, 4].  The loss is the negative log-likelihood of the target
(f, y1, y2) under the mixture:

  -log sum_k pi_k softmax(face logits_k)[f] N2(y1, y2 | mu1, mu2, s1, s2, rho).

Parameters are one flat FP64 vector in the order W1, b1, W2, b2, W3, b3, W4, b4 with every
W stored input-major ([in, out], row-major).  Forward, loss and backward are written with
numpy matrix products and elementwise operations, nothing fused.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

D_IN = 16
HID = 256
N_COMP = 16
N_FACE = 2
D_OUT = N_COMP * (1 + N_FACE + 5)     # 128
SHAPES = [(D_IN, HID), (HID,), (HID, HID), (HID,), (HID, HID), (HID,), (HID, D_OUT), (D_OUT,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))
LOGSIG_MIN, LOGSIG_MAX = -6.0, 4.0
RHO_SCALE = 0.95

O_PI, O_FACE, O_MU1, O_S1, O_MU2, O_S2, O_RHO = 0, 16, 48, 64, 80, 96, 112


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def _phi_cdf(z):
    return 0.5 * special.erfc(-z / math.sqrt(2.0))      # = (1 + erf(z / sqrt 2)) / 2, no cancellation


def gelu(z):
    return z * _phi_cdf(z)


def gelu_grad(z):
    return _phi_cdf(z) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, keep=False):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    z1 = X @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    z3 = h2 @ W3 + b3
    h3 = gelu(z3)
    o = h3 @ W4 + b4
    if keep:
        return o, (X, z1, h1, z2, h2, z3, h3)
    return o


def split(o):
    a = o[:, O_PI:O_PI + N_COMP]
    fl = o[:, O_FACE:O_FACE + 2 * N_COMP].reshape(-1, N_COMP, 2)
    mu1 = o[:, O_MU1:O_MU1 + N_COMP]
    s1 = np.clip(o[:, O_S1:O_S1 + N_COMP], LOGSIG_MIN, LOGSIG_MAX)
    mu2 = o[:, O_MU2:O_MU2 + N_COMP]
    s2 = np.clip(o[:, O_S2:O_S2 + N_COMP], LOGSIG_MIN, LOGSIG_MAX)
    rho = RHO_SCALE * np.tanh(o[:, O_RHO:O_RHO + N_COMP])
    return a, fl, mu1, s1, mu2, s2, rho


def component_logpdf(o, Y):
    """log of pi_k P(face | k) N2(y | k) per sample and component: (n, N_COMP)."""
    a, fl, mu1, s1, mu2, s2, rho = split(o)
    f = Y[:, 0].astype(np.int64)
    y1 = Y[:, 1][:, None]
    y2 = Y[:, 2][:, None]
    log_pi = a - special.logsumexp(a, axis=1, keepdims=True)
    log_pf = fl - special.logsumexp(fl, axis=2, keepdims=True)
    log_pf = np.take_along_axis(log_pf, f[:, None, None].repeat(N_COMP, axis=1), axis=2)[:, :, 0]
    z1 = (y1 - mu1) * np.exp(-s1)
    z2 = (y2 - mu2) * np.exp(-s2)
    om = 1.0 - rho * rho
    q = (z1 * z1 - 2.0 * rho * z1 * z2 + z2 * z2) / om
    log_n = -math.log(2.0 * math.pi) - s1 - s2 - 0.5 * np.log(om) - 0.5 * q
    return log_pi + log_pf + log_n


def nll(o, Y):
    """Per-sample negative log-likelihood."""
    return -special.logsumexp(component_logpdf(o, Y), axis=1)


def nll_grad_out(o, Y):
    """d(mean NLL)/d(o), written out from the definitions above."""
    n = o.shape[0]
    a, fl, mu1, s1, mu2, s2, rho = split(o)
    lc = component_logpdf(o, Y)
    w = np.exp(lc - special.logsumexp(lc, axis=1, keepdims=True))   # responsibilities
    f = Y[:, 0].astype(np.int64)
    y1 = Y[:, 1][:, None]
    y2 = Y[:, 2][:, None]
    g = np.zeros_like(o)
    pi = np.exp(a - special.logsumexp(a, axis=1, keepdims=True))
    g[:, O_PI:O_PI + N_COMP] = pi - w
    pf = np.exp(fl - special.logsumexp(fl, axis=2, keepdims=True))
    onehot = np.zeros_like(pf)
    onehot[np.arange(n), :, f] = 1.0
    g[:, O_FACE:O_FACE + 2 * N_COMP] = (w[:, :, None] * (pf - onehot)).reshape(n, -1)
    e1, e2 = np.exp(-s1), np.exp(-s2)
    z1 = (y1 - mu1) * e1
    z2 = (y2 - mu2) * e2
    om = 1.0 - rho * rho
    # q = (z1^2 - 2 rho z1 z2 + z2^2) / om ; log N = -s1 - s2 - log(om)/2 - q/2 + const
    dq_dz1 = (2.0 * z1 - 2.0 * rho * z2) / om
    dq_dz2 = (2.0 * z2 - 2.0 * rho * z1) / om
    dlogn_dmu1 = 0.5 * dq_dz1 * e1
    dlogn_dmu2 = 0.5 * dq_dz2 * e2
    dlogn_ds1 = -1.0 + 0.5 * dq_dz1 * z1
    dlogn_ds2 = -1.0 + 0.5 * dq_dz2 * z2
    q = (z1 * z1 - 2.0 * rho * z1 * z2 + z2 * z2) / om
    dq_drho = (-2.0 * z1 * z2) / om + q * (2.0 * rho) / om
    dlogn_drho = rho / om - 0.5 * dq_drho
    raw_rho = o[:, O_RHO:O_RHO + N_COMP]
    drho_draw = RHO_SCALE * (1.0 - np.tanh(raw_rho) ** 2)
    in1 = ((o[:, O_S1:O_S1 + N_COMP] > LOGSIG_MIN) & (o[:, O_S1:O_S1 + N_COMP] < LOGSIG_MAX)).astype(np.float64)
    in2 = ((o[:, O_S2:O_S2 + N_COMP] > LOGSIG_MIN) & (o[:, O_S2:O_S2 + N_COMP] < LOGSIG_MAX)).astype(np.float64)
    g[:, O_MU1:O_MU1 + N_COMP] = -w * dlogn_dmu1
    g[:, O_S1:O_S1 + N_COMP] = -w * dlogn_ds1 * in1
    g[:, O_MU2:O_MU2 + N_COMP] = -w * dlogn_dmu2
    g[:, O_S2:O_S2 + N_COMP] = -w * dlogn_ds2 * in2
    g[:, O_RHO:O_RHO + N_COMP] = -w * dlogn_drho * drho_draw
    return g / n


def loss_and_grad(theta, X, Y):
    """Mean NLL and its gradient with respect to theta (backpropagation)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    o, (X_, z1, h1, z2, h2, z3, h3) = forward(theta, X, keep=True)
    loss = float(nll(o, Y).mean())
    go = nll_grad_out(o, Y)
    gW4 = h3.T @ go
    gb4 = go.sum(axis=0)
    gz3 = (go @ W4.T) * gelu_grad(z3)
    gW3 = h2.T @ gz3
    gb3 = gz3.sum(axis=0)
    gz2 = (gz3 @ W3.T) * gelu_grad(z2)
    gW2 = h1.T @ gz2
    gb2 = gz2.sum(axis=0)
    gz1 = (gz2 @ W2.T) * gelu_grad(z1)
    gW1 = X.T @ gz1
    gb1 = gz1.sum(axis=0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def init(seed=0):
    """Glorot-uniform weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = math.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s))
        else:
            parts.append(np.zeros(s))
    return pack(parts)
