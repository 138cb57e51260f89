"""Plain FP64 CPU oracle for the data-driven model fits and the distance measure (TEST INFRASTRUCTURE).

Test infrastructure only, like the rest of ``oracle/``: imported by ``tests/``, never by the
product library, and sharing no code with it.

What it computes (paper: Methods, "Data-driven physically motivated models", "Technical details
regarding the parameter identification", and "Distance Measure"):

* Mixing orders (Eq. mix): row k of a 2D Lissajous system matrix is labelled by the integers
  (m_x, m_y) with k = m_x N_dens + m_y (N_dens + 1), taking the pair of smallest |m_x| + |m_y|
  (``mixing_order``), and the graded row set I_freq = {k(m_x, m_y) : 0 <= m_x <= M_x,
  0 <= m_y <= M_y} without (0, 0), (0, 1), (1, 0) (``frequency_index_set``).
* Models M0 / M1: for one dictionary element Phi_q (rows k, columns = the N offset positions) and
  the measured matrix S of one angle, the per-row complex scale a_k minimising
  || diag(a) Phi_q - S ||_F is a_k = S_k conj(Phi_{q;k})^T / ||Phi_{q;k}||^2 (``fit_scaling``).
* Eq. error1: per row, eps = (1/sqrt(N)) ||S_k - S^model_k||_2 / ||S_k||_inf (``nrmse_rows``);
  the per-frequency measure averages eps^2 over the angles (and, as the paper notes, also over the
  receive channels), the global measure averages eps_freq^2 over I_freq (Eq. globalMeasure).
"""
from __future__ import annotations

import numpy as np


def mixing_order(k, n_dens=16):
    """(m_x, m_y) with k = m_x n_dens + m_y (n_dens + 1) and the smallest |m_x| + |m_y|, found by
    brute force over every m_x with |m_x| <= 2|k| + 1 (the pair (-k, k) already has sum 2|k|, so a
    minimiser has |m_x| <= 2|k|).  The minimiser is asserted to be unique rather than assumed."""
    k = int(k)
    best, arg = None, []
    R = 2 * abs(k) + 1
    for mx in range(-R, R + 1):
        rest = k - mx * n_dens
        if rest % (n_dens + 1):
            continue
        my = rest // (n_dens + 1)
        s = abs(mx) + abs(my)
        if best is None or s < best:
            best, arg = s, [(mx, my)]
        elif s == best:
            arg.append((mx, my))
    assert len(arg) == 1, f"mixing order of {k} is not unique: {arg}"
    return arg[0]


def frequency_index_set(Mx, My, n_dens=16):
    """I_freq: k(m_x, m_y) for 0 <= m_x <= Mx, 0 <= m_y <= My without (0,0), (0,1), (1,0), in the
    order m_x-major (the paper does not order the set; sums over it do not depend on the order)."""
    out = []
    for mx in range(Mx + 1):
        for my in range(My + 1):
            if (mx, my) in ((0, 0), (0, 1), (1, 0)):
                continue
            out.append(mx * n_dens + my * (n_dens + 1))
    return np.array(out, dtype=np.int64)


def fit_scaling(Phi, S):
    """Closed-form per-row scale of models M0/M1: Phi, S complex [K, N] (row k = frequency,
    column = offset position).  Returns a [K] with a_k = S_k conj(Phi_k)^T / ||Phi_k||^2 (a row of
    Phi that is zero everywhere gets a_k = 0)."""
    Phi = np.asarray(Phi, complex)
    S = np.asarray(S, complex)
    num = np.sum(S * np.conj(Phi), axis=-1)
    den = np.sum(np.abs(Phi) ** 2, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def nrmse_rows(S, S_model):
    """Eq. error1 for every row: (1/sqrt(N)) ||S_k - S_model_k||_2 / ||S_k||_inf, arrays [..., N]."""
    S = np.asarray(S, complex)
    S_model = np.asarray(S_model, complex)
    N = S.shape[-1]
    return np.linalg.norm(S - S_model, axis=-1) / np.sqrt(N) / np.max(np.abs(S), axis=-1)


def eps_freq(eps):
    """Per-frequency NRMSE: eps [angles, channels, k] -> [k], the root mean square over angles and
    receive channels."""
    eps = np.asarray(eps, float)
    return np.sqrt(np.mean(eps ** 2, axis=(0, 1)))


def eps_global(eps_f):
    """Global NRMSE (Eq. globalMeasure): root mean square of eps_freq over the rows of I_freq."""
    eps_f = np.asarray(eps_f, float)
    return float(np.sqrt(np.mean(eps_f ** 2)))


def m1_measures(Phi, S, kset):
    """Model M1 for one parameter pair over all angles: Phi, S complex [angles, channels, bins, N]
    (bins indexed by k).  Fits a per (angle, channel, k) and returns (a [angles, channels, bins],
    eps rows [angles, channels, bins], eps_freq [len(kset)], eps_global)."""
    a = fit_scaling(Phi, S)
    eps = nrmse_rows(S, a[..., None] * Phi)
    ef = eps_freq(eps[:, :, kset])
    return a, eps, ef, eps_global(ef)


# --- model M2: weighted non-negative superposition with truncated-SVD regularisation -------------

def m2_system(Psi, S, kset):
    """Dictionary matrix and data of model M2 (Eq. LSfitM2 / LSfitM2_alternative).

    Psi [J, angles, channels, bins, N] complex: the scaled dictionary Psi_q = diag(a_q) Phi_q of every
    parameter pair j and angle; S [angles, channels, bins, N]: the measured matrices.  Rows are taken
    for the bins of kset (I_freq) and weighted by Sigma = 1 / ||S_{angle; channel, k}||_inf (the
    paper's weighting per frequency row, applied per receive channel).  Returns (M [R, J], y [R])
    with R = angles * channels * len(kset) * N, rows in that order, columns the pairs j."""
    Psi = np.asarray(Psi, complex)[:, :, :, kset, :]
    S = np.asarray(S, complex)[:, :, kset, :]
    w = 1.0 / np.max(np.abs(S), axis=-1)                     # [angles, channels, k]
    M = (Psi * w[None, ..., None]).reshape(Psi.shape[0], -1).T
    y = (S * w[..., None]).reshape(-1)
    return M, y


def m2_weights(M, y, s=None):
    """Non-negative weights of model M2: min over real w >= 0 of || U_s^H (M w - y) ||_2 with U_s the
    left singular vectors of the s largest singular values of M (Eq. approx_low_rank); s = None keeps
    every singular value (the plain weighted least-squares fit, Eq. LSfitM2).  The complex problem in
    real unknowns is solved as the real stacked system [Re; Im] by Lawson-Hanson NNLS (a library
    routine standing in for the paper's interior-point method; both find a minimiser of the same
    convex problem).  Returns (w, full residual ||M w - y||^2, reduced objective)."""
    from scipy.optimize import nnls
    U, sv, Vh = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(sv > sv[0] * 1e-13)) if sv.size else 0
    s = r if s is None else min(int(s), r)
    R = sv[:s, None] * Vh[:s]                    # U_s^H M
    c = U[:, :s].conj().T @ y                     # U_s^H y
    A = np.vstack([R.real, R.imag])
    rhs = np.concatenate([c.real, c.imag])
    w, res = nnls(A, rhs, maxiter=50 * A.shape[1])
    full = float(np.linalg.norm(M @ w - y) ** 2)
    return w, full, float(res ** 2)


def m2_model(Psi, w):
    """S_model of every angle: sum_j w_j Psi_j ([angles, channels, bins, N])."""
    return np.tensordot(np.asarray(w, float), np.asarray(Psi, complex), axes=(0, 0))
