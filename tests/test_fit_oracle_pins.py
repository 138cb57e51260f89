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
