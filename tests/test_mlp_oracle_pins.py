"""Pins of the FP64 network reference (oracle/mlp_oracle.py) against facts outside itself:
library routines (the normal CDF and density from scipy.stats), closed forms (GELU identities, the
first Adam step), a hand-computed one-unit network and central finite differences of the loss."""
import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle as O

M = O.mlp_oracle


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-6, 6, 121)
    assert np.abs(M.gelu(x) - x * norm.cdf(x)).max() < 1e-15
    # identity gelu(x) - gelu(-x) = x  (Phi(x) + Phi(-x) = 1)
    assert np.abs(M.gelu(x) - M.gelu(-x) - x).max() < 1e-14
    assert M.gelu(0.0) == 0.0
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15


def test_gelu_grad_matches_cdf_plus_density_and_fd():
    x = np.linspace(-5, 5, 101)
    assert np.abs(M.gelu_grad(x) - (norm.cdf(x) + x * norm.pdf(x))).max() < 1e-14
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.abs(fd - M.gelu_grad(x)).max() < 1e-8


def test_one_unit_network_by_hand():
    # z1 = 2 * 1 - 1 = 1, a1 = gelu(1) = Phi(1); y = 3 a1 + 0.5
    y, _ = M.forward([np.array([[2.0]]), np.array([[3.0]])], [np.array([-1.0]), np.array([0.5])], np.array([[1.0]]))
    assert abs(y[0, 0] - (3 * norm.cdf(1.0) + 0.5)) < 1e-15


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_central_differences(seed):
    widths = [8, 16, 12, 16, 10, 6]
    Ws, bs = M.init_params(widths, seed)
    r = np.random.default_rng(100 + seed)
    X = r.normal(size=(7, widths[0]))
    T = r.normal(size=(7, widths[-1]))
    y, cache = M.forward(Ws, bs, X)
    gW, gb = M.backward(Ws, cache, y, T)

    def L():
        return M.loss(M.forward(Ws, bs, X)[0], T)

    h = 1e-6
    for l in range(len(Ws)):
        for arr, g in ((Ws[l], gW[l]), (bs[l], gb[l])):
            flat = arr.reshape(-1)
            gf = g.reshape(-1)
            for idx in r.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = L()
                flat[idx] = old - h
                lm = L()
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gf[idx]) < 1e-7 * max(1.0, abs(gf[idx])) + 1e-9, (l, idx, fd, gf[idx])


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so the update is -lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    p0 = p.copy()
    m, v = np.zeros(4), np.zeros(4)
    M.adam_step([p], [g], [m], [v], 1, lr=0.01)
    assert np.allclose(p, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_minimises_a_quadratic():
    p = np.array([3.0, -2.0])
    m, v = np.zeros(2), np.zeros(2)
    for t in range(1, 3001):
        M.adam_step([p], [2 * (p - np.array([0.5, 1.5]))], [m], [v], t, lr=0.01)
    assert np.abs(p - np.array([0.5, 1.5])).max() < 1e-3


def test_loss_is_mean_square():
    y = np.array([[1.0, 2.0], [3.0, 4.0]])
    t = np.zeros((2, 2))
    assert M.loss(y, t) == (1 + 4 + 9 + 16) / 4
