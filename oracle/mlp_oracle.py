"""Plain FP64 CPU reference of the learned surrogate's network (TEST INFRASTRUCTURE).

Imported only by tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg; the
product library never calls it and shares no code with it.

The paper has no learned part: the network maps a particle instance (log D, sigma = K V / (k_B T),
alpha, easy axis n as a unit 3-vector, 2D offset field) to the real and imaginary parts of
the first harmonics of dm/dt (the phi-hat of model M1).  What is fixed here is ordinary
deep-learning arithmetic, written out plainly:

* a stack of affine layers z_l = W_l a_{l-1} + b_l, a_l = gelu(z_l) on every layer but the
  last (the last layer is affine only);
* gelu(x) = x * Phi(x) with Phi the standard normal CDF, Phi(x) = (1 + erf(x / sqrt 2)) / 2
  (the exact erf form, not the tanh approximation);
* loss = mean over all batch rows and outputs of (y - t)^2;
* the gradient by the chain rule (reverse accumulation), layer by layer;
* Adam (Kingma & Ba, 2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Weights use the row-major (out, in) convention.  Pins live in tests/test_mlp_oracle_pins.py.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    """x * Phi(x), exact erf form."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    """d gelu / dx = Phi(x) + x * phi(x), phi the standard normal density."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def init_params(widths, seed):
    """Weights ~ U(-1/sqrt(in), 1/sqrt(in)) (the usual default), biases likewise; FP64 lists."""
    r = np.random.default_rng(seed)
    Ws, bs = [], []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        s = 1.0 / math.sqrt(fan_in)
        Ws.append(r.uniform(-s, s, (fan_out, fan_in)))
        bs.append(r.uniform(-s, s, fan_out))
    return Ws, bs


def forward(Ws, bs, X):
    """Returns (y, cache): y [B, out]; cache holds the layer inputs and pre-activations."""
    a = np.asarray(X, dtype=np.float64)
    acts, pre = [a], []
    n = len(Ws)
    for l in range(n):
        z = a @ np.asarray(Ws[l], np.float64).T + np.asarray(bs[l], np.float64)
        pre.append(z)
        a = gelu(z) if l < n - 1 else z
        acts.append(a)
    return a, (acts, pre)


def loss(y, t):
    """Mean squared error over every element."""
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(Ws, cache, y, t):
    """Gradients of loss(y, t) with respect to every W_l and b_l (chain rule, last layer first)."""
    acts, pre = cache
    n = len(Ws)
    B_out = np.asarray(y).size
    dz = 2.0 * (np.asarray(y, np.float64) - np.asarray(t, np.float64)) / B_out
    gW, gb = [None] * n, [None] * n
    for l in range(n - 1, -1, -1):
        gW[l] = dz.T @ acts[l]
        gb[l] = dz.sum(axis=0)
        if l > 0:
            da = dz @ np.asarray(Ws[l], np.float64)
            dz = da * gelu_grad(pre[l - 1])
    return gW, gb


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of every array in `params` (in place); t is the 1-based step count."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= b1
        mm += (1.0 - b1) * g
        vv *= b2
        vv += (1.0 - b2) * g * g
        mhat = mm / (1.0 - b1 ** t)
        vhat = vv / (1.0 - b2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
