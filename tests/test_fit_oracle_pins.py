"""Pins of the fit / distance-measure oracle (oracle/fit_oracle.py) against what the paper and the
mathematics fix: hand-worked mixing orders of Eq. mix, an independent search by increasing order sum,
the least-squares optimality of the closed-form scale of models M0/M1 (library lstsq, exact recovery),
and hand-computed values of Eq. error1 and Eq. globalMeasure."""
import numpy as np
import pytest

from oracle import fit_oracle as F


@pytest.mark.parametrize("k,expect", [(0, (0, 0)), (16, (1, 0)), (17, (0, 1)), (33, (1, 1)), (1, (-1, 1)),
                                      (-1, (1, -1)), (32, (2, 0)), (50, (1, 2)), (15, (2, -1))])
def test_mixing_order_hand_values(k, expect):
    # Eq. mix with N_dens = 16: k = 16 m_x + 17 m_y; e.g. 15 = 16 * 2 + 17 * (-1)
    assert F.mixing_order(k) == expect
    mx, my = expect
    assert 16 * mx + 17 * my == k


def test_mixing_order_by_increasing_order_sum():
    """Independent search: enumerate (m_x, m_y) by |m_x| + |m_y| = 0, 1, 2, ...; the first sum that
    reaches k must hold exactly one pair, and it must be the oracle's."""
    for k in range(-300, 301):
        s = 0
        while True:
            hits = [(mx, sgn * (s - abs(mx))) for mx in range(-s, s + 1) for sgn in ((1, -1) if s - abs(mx) else (1,))
                    if 16 * mx + 17 * sgn * (s - abs(mx)) == k]
            if hits:
                assert hits == [F.mixing_order(k)], (k, hits)
                break
            s += 1


def test_frequency_index_set():
    ks = F.frequency_index_set(3, 4)
    assert len(ks) == 4 * 5 - 3 and len(set(ks.tolist())) == len(ks)
    assert 0 not in ks and 16 not in ks and 17 not in ks and 33 in ks and 3 * 16 + 4 * 17 in ks
    for k in ks:
        mx, my = F.mixing_order(k)
        assert 0 <= mx <= 3 and 0 <= my <= 4


def test_fit_scaling_recovers_exact_scale_and_is_least_squares():
    r = np.random.default_rng(1)
    K, N = 7, 121
    Phi = r.normal(size=(K, N)) + 1j * r.normal(size=(K, N))
    a = r.normal(size=K) + 1j * r.normal(size=K)
    assert np.allclose(F.fit_scaling(Phi, a[:, None] * Phi), a, rtol=1e-13, atol=0)
    S = r.normal(size=(K, N)) + 1j * r.normal(size=(K, N))
    ah = F.fit_scaling(Phi, S)
    for k in range(K):
        ref = np.linalg.lstsq(Phi[k][:, None], S[k], rcond=None)[0][0]
        assert abs(ah[k] - ref) <= 1e-12 * abs(ref)
        # the residual is orthogonal to the dictionary row
        assert abs(np.vdot(Phi[k], S[k] - ah[k] * Phi[k])) <= 1e-10 * np.linalg.norm(S[k]) * np.linalg.norm(Phi[k])
    z = np.zeros((1, N))
    assert F.fit_scaling(z, S[:1])[0] == 0


def test_nrmse_hand_values():
    S = np.array([[3.0, -4j]])
    assert F.nrmse_rows(S, np.zeros_like(S))[0] == pytest.approx(np.sqrt(25 / 2) / 4, rel=1e-15)
    assert F.nrmse_rows(S, S)[0] == 0.0
    # rows normalised by their own infinity norm: scaling a row leaves its error unchanged
    S2 = np.array([[1.0, 2.0, -2.0], [100.0, 200.0, -200.0]])
    M2 = S2 * 1.1
    e = F.nrmse_rows(S2, M2)
    assert e[0] == pytest.approx(e[1], rel=1e-14)
    assert e[0] == pytest.approx(0.1 * 3 / np.sqrt(3) / 2, rel=1e-14)


def test_frequency_and_global_measures_hand_values():
    eps = np.zeros((2, 2, 3))
    eps[0, 0] = [0.1, 0.2, 0.0]
    eps[1, 1] = [0.1, 0.0, 0.4]
    ef = F.eps_freq(eps)
    assert np.allclose(ef, [np.sqrt(0.02 / 4), np.sqrt(0.04 / 4), np.sqrt(0.16 / 4)], rtol=1e-15)
    assert F.eps_global(ef) == pytest.approx(np.sqrt((0.02 + 0.04 + 0.16) / 12), rel=1e-15)
    assert F.eps_global(np.full(5, 0.3)) == pytest.approx(0.3, rel=1e-15)


def test_m1_measures_vanish_at_the_generating_parameters():
    r = np.random.default_rng(2)
    Phi = r.normal(size=(3, 2, 40, 25)) + 1j * r.normal(size=(3, 2, 40, 25))
    a = np.exp(1j * np.linspace(0, 2, 40)) * (1 + 0.1 * np.arange(40))
    S = a[None, None, :, None] * Phi
    kset = F.frequency_index_set(1, 1)
    ah, eps, ef, eg = F.m1_measures(Phi, S, kset)
    assert np.allclose(ah, np.broadcast_to(a, ah.shape), rtol=1e-13)
    assert eg < 1e-14
    _, _, _, eg2 = F.m1_measures(Phi + 0.1 * r.normal(size=Phi.shape), S, kset)
    assert eg2 > 1e-3


def test_m2_system_layout_and_weighting_by_hand():
    # one pair, two angles, one channel, bins 0..2 (kset = [1, 2]), two positions
    Psi = np.zeros((1, 2, 1, 3, 2), complex)
    Psi[0, 0, 0, 1] = [1.0, 2.0]
    Psi[0, 1, 0, 2] = [3j, 0.0]
    S = np.zeros((2, 1, 3, 2), complex)
    S[0, 0, 1] = [4.0, -2.0]     # ||.||_inf = 4
    S[0, 0, 2] = [1.0, 1.0]      # 1
    S[1, 0, 1] = [0.5, 0.0]      # 0.5
    S[1, 0, 2] = [0.0, 2.0]      # 2
    M, y = F.m2_system(Psi, S, np.array([1, 2]))
    assert M.shape == (8, 1)
    # rows: angle 0 (k = 1: pos 0, 1; k = 2: pos 0, 1), angle 1 (...)
    assert np.allclose(M[:, 0], [1 / 4, 2 / 4, 0, 0, 0, 0, 3j / 2, 0])
    assert np.allclose(y, [1, -0.5, 1, 1, 1, 0, 0, 1])


def test_m2_weights_recover_a_nonnegative_superposition():
    r = np.random.default_rng(4)
    M = r.normal(size=(60, 6)) + 1j * r.normal(size=(60, 6))
    w_true = np.array([0.0, 1.5, 0.0, 0.3, 2.0, 0.0])
    w, full, red = F.m2_weights(M, M @ w_true)
    assert np.allclose(w, w_true, atol=1e-10)
    assert full < 1e-18


def test_m2_weights_equal_least_squares_when_interior_and_satisfy_kkt():
    r = np.random.default_rng(5)
    M = r.normal(size=(80, 5)) + 1j * r.normal(size=(80, 5))
    w_pos = np.array([1.0, 2.0, 0.5, 1.5, 0.8])
    y = M @ w_pos + 0.01 * (r.normal(size=80) + 1j * r.normal(size=80))
    w, _, _ = F.m2_weights(M, y)
    ref = np.linalg.lstsq(np.vstack([M.real, M.imag]), np.concatenate([y.real, y.imag]), rcond=None)[0]
    assert (ref > 0).all() and np.allclose(w, ref, rtol=1e-10)
    # active constraints: KKT of min ||M w - y||^2 over w >= 0
    y2 = M @ np.array([1.0, -1.0, 0.5, -0.2, 0.8]) + 0.05 * r.normal(size=80)
    w2, _, _ = F.m2_weights(M, y2)
    g = np.real(M.conj().T @ (M @ w2 - y2))
    assert (w2 >= 0).all() and (w2 == 0).any()
    assert np.all(np.abs(g[w2 > 0]) < 1e-9 * np.abs(g).max() + 1e-12)
    assert np.all(g[w2 == 0] > -1e-9 * np.abs(g).max())


def test_m2_truncation_keeping_every_singular_value_is_the_plain_fit():
    r = np.random.default_rng(6)
    M = r.normal(size=(50, 7)) + 1j * r.normal(size=(50, 7))
    y = r.normal(size=50) + 1j * r.normal(size=50)
    w0, full0, red0 = F.m2_weights(M, y)
    w1, full1, red1 = F.m2_weights(M, y, s=7)
    U = np.linalg.svd(M, full_matrices=False)[0]
    out = np.linalg.norm(y - U @ (U.conj().T @ y)) ** 2
    assert np.allclose(w0, w1, atol=1e-12) and abs(full0 - (red1 + out)) < 1e-9 * full0
    # a stronger truncation cannot lower the full residual below the untruncated optimum
    w3, full3, _ = F.m2_weights(M, y, s=3)
    assert full3 >= full0 * (1 - 1e-12)
