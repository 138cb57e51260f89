"""CPU-only checks of the C-ABI library: it loads, exports every declared symbol, and
its host-built operator tables agree with the oracle's independent assembly."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpn.h")

fpn = pytest.importorskip("paper_2106_08040_amd")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpn_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(fpn.LIB_PATH)
    names = declared_functions()
    assert "fpn_solve" in names and "fpn_stationary" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(fpn.EXPORTED) == names


@pytest.mark.parametrize("L,seed", [(2, 0), (6, 1), (10, 2), (16, 3)])
def test_host_operator_matches_oracle_assembly(L, seed):
    """Library tables (algebraic construction in the easy-axis frame) vs the oracle's direct
    quadrature of the weak form with n = z: entry-wise to 1e-11 of the largest entry."""
    r = np.random.default_rng(seed)
    p = dict(D=r.uniform(14e-9, 28e-9), Ms=r.uniform(3e5, 5e5), K=r.uniform(0, 1e4), alpha=r.uniform(0.05, 0.4),
             T=r.uniform(250, 320))
    h = r.normal(size=3) * 6e-3
    A = fpn.fpn_host_operator(L, p["D"], p["Ms"], p["K"], p["alpha"], p["T"], h)
    A0, Aa, _ = O.operator_parts(p, [0.0, 0.0, 1.0], L)
    Ao = A0 + h[0] * Aa[0] + h[1] * Aa[1] + h[2] * Aa[2]
    scale = np.abs(Ao).max()
    assert np.abs(A - Ao).max() < 1e-11 * scale


def test_frame_is_a_rotation_onto_the_easy_axis():
    r = np.random.default_rng(5)
    for _ in range(20):
        n = r.normal(size=3)
        n /= np.linalg.norm(n)
        R = fpn.fpn_host_frame(n)
        assert np.allclose(R @ np.array([0, 0, 1.0]), n, atol=1e-14)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
    for n in ([1, 0, 0], [0, 1, 0], [0, 0, -1]):
        R = fpn.fpn_host_frame(n)
        assert np.allclose(R[:, 2], n)


def test_host_argument_errors():
    with pytest.raises(fpn.FpnError) as e:
        fpn.fpn_host_operator(0, 20e-9, 474e3, 2e3, 0.1, 295.0, [0, 0, 0])
    assert e.value.code == fpn.FPN_E_RANGE
    with pytest.raises(fpn.FpnError) as e:
        fpn.fpn_host_operator(4, -1.0, 474e3, 2e3, 0.1, 295.0, [0, 0, 0])
    assert e.value.code == fpn.FPN_E_ARG
    with pytest.raises(fpn.FpnError) as e:
        fpn.fpn_host_frame([1.0, 1.0, 0.0])
    assert e.value.code == fpn.FPN_E_ARG
    assert fpn.fpn_host_table_nnz(0) == -1
    assert fpn.fpn_status_string(fpn.FPN_E_DEVICE) == "HIP device error"


def test_table_sizes_and_selection_rules():
    for L in (4, 10, 16):
        nnz = fpn.fpn_host_table_nnz(L)
        N = (L + 1) ** 2
        assert 10 * N < nnz < 30 * N
        # row 0 of the operator vanishes (probability conservation) and couplings stay within |dl| <= 2
        A = fpn.fpn_host_operator(L, 20e-9, 474e3, 2e3, 0.1, 295.0, [3e-3, -2e-3, 1e-3])
        assert np.abs(A[0]).max() == 0.0
        ls = O.sh_degrees(L)
        far = np.abs(ls[:, None] - ls[None, :]) > 2
        assert np.abs(A[far]).max() == 0.0


def test_stepper_wave_options():
    """Workgroup sizes compiled per degree: 8, 12, 16 up to L = 13, 8 up to 16, one wide layout above."""
    import paper_2106_08040_amd as fpn
    for L in range(1, 14):
        assert fpn.fpn_stepper_wave_options(L) == [8, 12, 16]
    for L in (14, 15, 16):
        assert fpn.fpn_stepper_wave_options(L) == [8]
    for L in range(17, 25):
        assert fpn.fpn_stepper_wave_options(L) == [0]
    for L in (0, 25):
        with pytest.raises(fpn.FpnError):
            fpn.fpn_stepper_wave_options(L)


def test_mixing_orders_and_frequency_set_match_oracle_bit_exact():
    """fpn_mixing_order / fpn_frequency_index_set (host integer code) against the oracle's brute force."""
    import paper_2106_08040_amd as fpn
    from oracle import fit_oracle as F
    for n in (16, 5, 31):
        for k in range(-700, 701):
            assert fpn.mixing_order(k, n) == F.mixing_order(k, n), (k, n)
    for Mx, My in ((0, 0), (1, 1), (6, 9), (12, 11)):
        assert np.array_equal(fpn.frequency_index_set(Mx, My), F.frequency_index_set(Mx, My).astype(np.int32))
    with pytest.raises(fpn.FpnError):
        fpn.mixing_order(5, 0)


@pytest.mark.parametrize("s", [0, 3, 6])
def test_m2_weights_match_oracle(s):
    """fpn_m2_weights (host: Hermitian Jacobi eigenvectors of G = M^H M, interior point) against the
    oracle (SVD of M, Lawson-Hanson NNLS) on a random complex dictionary with active constraints: the
    truncated objective (the quantity the paper minimises) agrees; untruncated, the minimiser is unique
    and the weights agree too."""
    import paper_2106_08040_amd as fpn
    from oracle import fit_oracle as F
    r = np.random.default_rng(20 + s)
    M = r.normal(size=(300, 9)) + 1j * r.normal(size=(300, 9))
    M[:, 1] = M[:, 0] * 0.9 + 0.1 * M[:, 1]     # nearly dependent columns, as in a fine dictionary
    y = M @ np.array([1.0, 0.0, 0.5, 0.0, 2.0, 0.3, 0.0, 0.0, 1.0]) + 0.3 * (r.normal(size=300) + 1j * r.normal(size=300))
    G, b, yy = M.conj().T @ M, M.conj().T @ y, float(np.vdot(y, y).real)
    w, full, red, rank = fpn.m2_weights(G, b, yy, s=s)
    wo, fullo, redo = F.m2_weights(M, y, s=None if s == 0 else s)
    assert rank == (9 if s == 0 else s)
    assert (w >= 0).all()
    assert abs(red - redo) <= 1e-9 * yy
    assert abs(full - float(np.linalg.norm(M @ w - y) ** 2)) <= 1e-9 * full
    if s == 0:
        assert np.allclose(w, wo, atol=1e-6 * wo.max())
