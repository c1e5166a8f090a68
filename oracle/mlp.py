"""Float64 reference of the error surrogate network (oracle).  Test
infrastructure only.

The surrogate maps a point-set description (c1, c2, m, r) to the predicted
log10 of the float32 Winograd error, so that the smooth error curve the paper
observes (Section 6.1) can be searched with few exact evaluations.  Nothing in
the paper fixes the network; this module defines it plainly:

  features f = (ln c1 / ln 20, ln c2 / ln 20, (m - 5) / 3, r - 4)
  h1 = gelu(W1 f + b1), h2 = gelu(W2 h1 + b2), h3 = gelu(W3 h2 + b3)
  out = W4 h3 + b4                    widths 4 -> 128 -> 128 -> 128 -> 1
  gelu(z) = z * Phi(z) = z (1 + erf(z / sqrt 2)) / 2     (exact erf form)
  loss = mean over the batch of (out - target)^2
  Adam (Kingma and Ba, 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Gradients are derived by hand (chain rule); the tests pin them with central
finite differences.
"""
from __future__ import annotations

import math

import numpy as np

F64 = np.float64
WIDTHS = (4, 128, 128, 128, 1)
LN20 = math.log(20.0)


def features(c1, c2, m, r):
    """Input encoding (B, 4) in float64."""
    c1 = np.asarray(c1, dtype=F64)
    c2 = np.asarray(c2, dtype=F64)
    m = np.asarray(m, dtype=F64)
    r = np.asarray(r, dtype=F64)
    return np.stack([np.log(c1) / LN20, np.log(c2) / LN20, (m - 5.0) / 3.0, r - 4.0], axis=1)


_erf = np.vectorize(math.erf, otypes=[F64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * pdf


def forward(params, X):
    """Returns (out (B,), cache) for params = [(W (out,in), b (out,)), ...]."""
    a = np.asarray(X, dtype=F64)
    cache = []
    for li, (W, b) in enumerate(params):
        W = np.asarray(W, dtype=F64)
        b = np.asarray(b, dtype=F64)
        z = a @ W.T + b
        cache.append((a, z))
        a = gelu(z) if li < len(params) - 1 else z
    return a[:, 0], cache


def loss_and_grads(params, X, target):
    """Mean squared error and its gradient with respect to every W and b."""
    out, cache = forward(params, X)
    t = np.asarray(target, dtype=F64)
    B = out.shape[0]
    diff = out - t
    loss = float(np.mean(diff * diff))
    dz = (2.0 / B) * diff[:, None]              # d loss / d out
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        a_in, z = cache[li]
        if li < len(params) - 1:
            dz = dz * gelu_grad(z)
        W = np.asarray(params[li][0], dtype=F64)
        grads[li] = (dz.T @ a_in, dz.sum(axis=0))
        dz = dz @ W
    return loss, grads


def adam_step(params, grads, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  state is a list of (m_W, v_W, m_b,
    v_b) float64 arrays, updated in place; returns the new params."""
    new = []
    for (W, b), (gW, gb), st in zip(params, grads, state):
        outp = []
        for idx, (p, gr) in enumerate(((W, gW), (b, gb))):
            mo, vo = st[2 * idx], st[2 * idx + 1]
            mo[...] = b1 * mo + (1 - b1) * gr
            vo[...] = b2 * vo + (1 - b2) * gr * gr
            mhat = mo / (1 - b1 ** t)
            vhat = vo / (1 - b2 ** t)
            outp.append(np.asarray(p, dtype=F64) - lr * mhat / (np.sqrt(vhat) + eps))
        new.append((outp[0], outp[1]))
    return new


def zero_state(params):
    return [(np.zeros_like(W, dtype=F64), np.zeros_like(W, dtype=F64),
             np.zeros_like(b, dtype=F64), np.zeros_like(b, dtype=F64)) for W, b in params]


def flatten(params):
    return np.concatenate([np.concatenate([np.ravel(W), np.ravel(b)]) for W, b in params])
