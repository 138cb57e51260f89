"""Plain FP64 CPU oracle for the Neel-rotation Fokker-Planck model (TEST INFRASTRUCTURE).

This module is test infrastructure only.  It may be imported by ``tests/``,
by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``;
the product library never imports, links or calls it, and it shares no code,
table or constant with the HIP path.

What it computes (paper: Methods, "Particle magnetization model"):

* Mean moment m(t) = integral over the unit sphere of m f(m, t)   (Eq. mean_magmom_FP),
  reported dimensionless (divided by m0 = V_C M_S, as the paper's phi-hat is).
* f solves the convection-diffusion equation on the sphere          (Eq. FP-general)
      df/dt = div(grad f)/(2 tau) - div(b f)
  with the Neel drift b(m, H, n) of Eq. convection and the constants
  p1..p4, tau, gamma-tilde listed right after it.
* Signal harmonics of dm/dt over one drive period                    (Eq. MPI_model_fourier,
  the phi-hat definition under model M1).

Discretisation (the paper solves with finite volumes; here a real
spherical-harmonic Galerkin expansion of degree <= L is used, which converges
to the same PDE solution):

* Real orthonormal spherical harmonics without Condon-Shortley phase,
  index i = l*l + l + m, m > 0 -> cos(m phi), m < 0 -> sin(|m| phi).
  Built from scipy's complex harmonics (a library primitive).
* Galerkin matrix (weak form, integration by parts on the closed sphere):
      dc_i/dt = sum_j A_ij c_j,
      A_ij = [ -l_i(l_i+1) delta_ij + int (grad Y_i . 2 tau b) Y_j ] / (2 tau)
  assembled directly from the drift of Eq. convection by exact product
  quadrature (Gauss-Legendre in cos(theta) x uniform phi).
* Initial state: the stationary density of the field at t = 0 with total
  probability one (the paper is silent on the initial condition).
* Time integration: 3-stage Radau IIA collocation (order 5, L-stable) on a
  uniform grid with r steps per sample interval, dense LU per step.
* Harmonics: Phi_k = (2 pi i k / T) * (1/N_s) sum_j m(t_j) exp(-2 pi i j k / N_s),
  i.e. the period integral of dm/dt e^{-2 pi i t k / T} taken exactly by parts
  (m is T-periodic) and the remaining integral of m by the rectangle rule.
  The rectangle rule applied to sampled dm/dt (RHS evaluation) is also
  returned as a diagnostic (``Phi_rect``).
* Equilibrium model (model M0, Eq. Langevin), the paper's baseline: the Langevin
  moment of the instantaneous field on the same samples and harmonics
  (``equilibrium_instance``).

Parity pins for every function live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.special as sps

# --- physical constants: the paper gives no values; CODATA 2018 values, mu0 = 4 pi 1e-7 ---
MU0 = 4e-7 * np.pi                 # vacuum permeability [T m / A]
KB = 1.380649e-23                  # Boltzmann constant [J / K]
GAMMA_E = 1.76085963023e11         # electron gyromagnetic ratio [rad / (s T)]


def particle_scalars(D, Ms, K, alpha, T):
    """Scalars of the Neel model (paper: constants after Eq. convection and in M0).

    V_C = pi D^3 / 6, gamma~ = gamma / (1 + alpha^2),
    tau = V_C M_S / (2 k_B T_B gamma~ alpha), beta = mu0 V_C M_S / (k_B T_B),
    sigma = K V_C / (k_B T_B).  ``beta_T`` is beta per tesla of mu0*H
    (beta * H with H = B / mu0), so beta_T * B is dimensionless.
    """
    V = np.pi * D ** 3 / 6.0
    gt = GAMMA_E / (1.0 + alpha ** 2)
    tau = V * Ms / (2.0 * KB * T * gt * alpha)
    beta_T = V * Ms / (KB * T)
    sigma = K * V / (KB * T)
    return dict(V=V, m0=V * Ms, gamma_t=gt, tau=tau, beta_T=beta_T, sigma=sigma,
                p1=gt * MU0, p2=gt * alpha * MU0, p3=2 * gt * K / Ms, p4=alpha * 2 * gt * K / Ms)


def sh_index(l, m):
    """Flat index of the real harmonic (l, m): i = l*l + l + m."""
    return l * l + l + m


def sh_degrees(L):
    """Degree l of every flat index 0..(L+1)^2-1."""
    return np.array([l for l in range(L + 1) for _ in range(-l, l + 1)])


def quadrature(nt, nph):
    """Product rule on the sphere: Gauss-Legendre in cos(theta), uniform in phi.

    Exact for spherical polynomials of degree <= min(2 nt - 1, nph - 1).
    Returns (theta, phi, weights), flattened.
    """
    x, wx = np.polynomial.legendre.leggauss(nt)
    th = np.arccos(x)
    ph = 2 * np.pi * np.arange(nph) / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = (wx[:, None] * np.full(nph, 2 * np.pi / nph)[None, :]).ravel()
    return TH.ravel(), PH.ravel(), W


def unit_vectors(theta, phi):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    m = np.stack([st * cp, st * sp, ct], 1)
    e_th = np.stack([ct * cp, ct * sp, -st], 1)
    e_ph = np.stack([-sp, cp, 0 * st], 1)
    return m, e_th, e_ph


def real_sh(L, theta, phi):
    """Real orthonormal harmonics and their surface gradients at points.

    Returns Y [N, Q] and G [N, Q, 3] (Cartesian components of grad_S Y).
    Built from scipy's complex harmonics (with Condon-Shortley phase, removed
    here) and their theta/phi derivatives.  Points must avoid the poles.
    """
    N = (L + 1) ** 2
    m_vec, e_th, e_ph = unit_vectors(theta, phi)
    st = np.sin(theta)
    Y = np.zeros((N, theta.size))
    G = np.zeros((N, theta.size, 3))
    for l in range(L + 1):
        for m in range(l + 1):
            y, dy = sps.sph_harm_y(l, m, theta, phi, diff_n=1)
            dth, dph = dy[..., 0], dy[..., 1]
            if m == 0:
                Y[sh_index(l, 0)] = y.real
                G[sh_index(l, 0)] = dth.real[:, None] * e_th + (dph.real / st)[:, None] * e_ph
            else:
                f = np.sqrt(2.0) * (-1) ** m
                Y[sh_index(l, m)] = f * y.real
                Y[sh_index(l, -m)] = f * y.imag
                G[sh_index(l, m)] = f * (dth.real[:, None] * e_th + (dph.real / st)[:, None] * e_ph)
                G[sh_index(l, -m)] = f * (dth.imag[:, None] * e_th + (dph.imag / st)[:, None] * e_ph)
    return Y, G


def galerkin_components(L, n):
    """Instance-independent Galerkin pieces for easy axis ``n`` (lab frame).

    With v = 2 tau b written through Phi = beta H.m + sigma (n.m)^2 as
    v = grad_S Phi - m x grad_S Phi / alpha (equivalent to Eq. convection
    with the listed p1..p4), the matrix is
        2 tau A = diag(lam) + sigma (Gd + Gp / alpha)
                  + sum_a beta H_a (Fd[a] + Fp[a] / alpha).
    Every piece is int (grad Y_i . w) Y_j for the vector field w named below.
    """
    n = np.asarray(n, float)
    th, ph, W = quadrature(L + 6, 2 * L + 12)
    Y, G = real_sh(L, th, ph)
    mv, _, _ = unit_vectors(th, ph)
    nm = mv @ n

    def proj(w):
        return (np.einsum("iqa,qa->iq", G, w) * W) @ Y.T

    e = np.eye(3)
    Fd = [proj(e[a][None, :] - mv[:, a:a + 1] * mv) for a in range(3)]          # grad_S (m_a)
    Fp = [proj(-np.cross(mv, e[a][None, :])) for a in range(3)]                 # -m x e_a
    Gd = proj(2 * nm[:, None] * (n[None, :] - nm[:, None] * mv))                # grad_S (n.m)^2
    Gp = proj(-2 * nm[:, None] * np.cross(mv, n[None, :]))                      # -m x grad (n.m)^2
    ls = sh_degrees(L)
    return dict(lam=-ls * (ls + 1.0), Fd=Fd, Fp=Fp, Gd=Gd, Gp=Gp)


def operator_parts(p, n, L):
    """A(t) = A0 + sum_a B_a(t) Aa[a] in 1/s, with B(t) = mu0 H(t) in tesla.

    ``p`` holds D, Ms, K, alpha, T (SI units); ``n`` is the easy axis.
    """
    sc = particle_scalars(p["D"], p["Ms"], p["K"], p["alpha"], p["T"])
    comp = galerkin_components(L, n)
    a = p["alpha"]
    inv2tau = 1.0 / (2.0 * sc["tau"])
    A0 = (np.diag(comp["lam"]) + sc["sigma"] * (comp["Gd"] + comp["Gp"] / a)) * inv2tau
    Aa = [sc["beta_T"] * (comp["Fd"][k] + comp["Fp"][k] / a) * inv2tau for k in range(3)]
    return A0, Aa, sc


def drive_field(drive, offset, t):
    """mu0 H(t) [T] = offset + amp * cos(2 pi freq t + phase), per lab axis (Eq. complete-problem's H = H_SF + H_DF)."""
    t = np.asarray(t, float)
    amp = np.asarray(drive["amp"], float)
    fr = np.asarray(drive["freq"], float)
    ph = np.asarray(drive.get("phase", (0.0, 0.0, 0.0)), float)
    return np.asarray(offset, float) + amp * np.cos(2 * np.pi * fr * t[..., None] + ph)


def stationary(A):
    """Null vector of A with c_00 = 1/sqrt(4 pi) (total probability 1): drop row 0, solve."""
    N = A.shape[0]
    c = np.zeros(N)
    c[0] = 1.0 / np.sqrt(4.0 * np.pi)
    c[1:] = np.linalg.solve(A[1:, 1:], -A[1:, 0] * c[0])
    return c


def moment(c):
    """<m> = int m f = sqrt(4 pi / 3) (c_{1,1}, c_{1,-1}, c_{1,0})  (Eq. mean_magmom_FP / m0)."""
    c = np.asarray(c)
    return np.sqrt(4 * np.pi / 3) * c[..., [3, 1, 2]]


# 3-stage Radau IIA collocation (nodes are the right Radau points on [0, 1]).
_S6 = np.sqrt(6.0)
RADAU_C = np.array([(4 - _S6) / 10, (4 + _S6) / 10, 1.0])
RADAU_A = np.array([[(88 - 7 * _S6) / 360, (296 - 169 * _S6) / 1800, (-2 + 3 * _S6) / 225],
                    [(296 + 169 * _S6) / 1800, (88 + 7 * _S6) / 360, (-2 - 3 * _S6) / 225],
                    [(16 - _S6) / 36, (16 + _S6) / 36, 1.0 / 9]])


def radau_step(Afun, t, y, h):
    """One Radau IIA step for the linear ODE y' = A(t) y: solve the 3N stage system, return Y_3."""
    N = y.size
    As = [Afun(t + c * h) for c in RADAU_C]
    M = np.eye(3 * N)
    for i in range(3):
        for j in range(3):
            M[i * N:(i + 1) * N, j * N:(j + 1) * N] -= h * RADAU_A[i, j] * As[j]
    Y = sla.lu_solve(sla.lu_factor(M, check_finite=False), np.tile(y, 3), check_finite=False)
    return Y[2 * N:]


def integrate_samples(Afun, c0, period, n_samples, settle, r, t0=0.0):
    """Integrate from c0 at t0 over (settle + 1) periods with r Radau steps per sample.

    Returns the states at t_j = t0 + settle*T + j T / N_s, j = 0..N_s-1.
    """
    h = period / (n_samples * r)
    y = np.array(c0, float)
    out = np.zeros((n_samples, y.size))
    first = settle * n_samples * r
    for step in range((settle + 1) * n_samples * r):
        if step >= first and (step - first) % r == 0:
            out[(step - first) // r] = y
        y = radau_step(Afun, t0 + step * h, y, h)
    return out


def harmonics_from_samples(m, period, n_harm):
    """Phi_k = (2 pi i k / T) (1/N_s) sum_j m_j e^{-2 pi i j k / N_s}, k = 0..n_harm; m is [N_s, ch]."""
    Ns = m.shape[0]
    j = np.arange(Ns)
    k = np.arange(n_harm + 1)
    E = np.exp(-2j * np.pi * np.outer(k, j) / Ns)          # direct sum, no FFT
    Mk = E @ m / Ns
    return (2j * np.pi * k / period)[:, None] * Mk


def solve_instance(p, n, L, drive, n_samples, settle, n_harm, r=2, offset=(0, 0, 0)):
    """Full procedure for one instance: stationary start at t = 0, Radau with r steps/sample.

    Returns dict with m [N_s, 3] (lab frame), Phi [n_harm+1, 3] complex,
    mdot [N_s, 3] (RHS-evaluated derivative) and Phi_rect (its rectangle-rule DFT).
    """
    A0, Aa, sc = operator_parts(p, n, L)
    offset = np.asarray(offset, float)

    def Afun(t):
        B = drive_field(drive, offset, t)
        return A0 + B[0] * Aa[0] + B[1] * Aa[1] + B[2] * Aa[2]

    c0 = stationary(Afun(0.0))
    T = drive["period"]
    cs = integrate_samples(Afun, c0, T, n_samples, settle, r)
    ts = settle * T + np.arange(n_samples) * T / n_samples
    m = moment(cs)
    mdot = np.array([moment(Afun(t) @ c) for t, c in zip(ts, cs)])
    Phi = harmonics_from_samples(m, T, n_harm)
    Ns = n_samples
    k = np.arange(n_harm + 1)
    Phi_rect = np.exp(-2j * np.pi * np.outer(k, np.arange(Ns)) / Ns) @ mdot / Ns
    return dict(m=m, Phi=Phi, mdot=mdot, Phi_rect=Phi_rect, c_last=cs[-1], r=r, scalars=sc)


# --- closed forms used by the pins -------------------------------------------------

def langevin(x):
    """L(x) = coth(x) - 1/x (paper Eq. Langevin with beta z -> x); series near 0."""
    x = np.asarray(x, float)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    return np.where(small, x / 3 - x ** 3 / 45, 1 / np.tanh(xs) - 1 / xs)


def peak_field(drive, offset, n_samples):
    """mu0 H(t_j) at t_j = j T / N_s of largest magnitude (the first sample within a relative 1e-9 of
    the largest squared magnitude)."""
    T = drive["period"]
    B = drive_field(drive, np.asarray(offset, float), np.arange(n_samples) * T / n_samples)
    b2 = np.einsum("ij,ij->i", B, B)
    return B[int(np.nonzero(b2 >= b2.max() * (1.0 - 1e-9))[0][0])]


def truncation_estimate(p, n, L, drive, offset, n_samples):
    """Estimate of the truncation error of degree L: |m_L - m_{L-2}| of the stationary moments under
    the largest sampled field (a heuristic indicator, not from the paper; the tests check that it
    bounds the degree-L error of the periodic m(t) against finite-volume and higher-degree solves)."""
    B = peak_field(drive, offset, n_samples)
    ms = []
    for LL in (L, L - 2):
        A0, Aa, _ = operator_parts(p, n, LL)
        ms.append(moment(stationary(A0 + B[0] * Aa[0] + B[1] * Aa[1] + B[2] * Aa[2])))
    return float(np.linalg.norm(ms[0] - ms[1]))


def select_degree(p, n, L_min, drive, offset, n_samples, tol, L_max=24):
    """Smallest degree L in L_min..L_max with truncation_estimate(L) <= tol (L_max if none); returns
    (L, its estimate)."""
    B = peak_field(drive, offset, n_samples)
    ms = {}

    def m_at(LL):
        if LL not in ms:
            A0, Aa, _ = operator_parts(p, n, LL)
            ms[LL] = moment(stationary(A0 + B[0] * Aa[0] + B[1] * Aa[1] + B[2] * Aa[2]))
        return ms[LL]

    for L in range(L_min, L_max + 1):
        e = float(np.linalg.norm(m_at(L) - m_at(L - 2)))
        if e <= tol:
            return L, e
    return L_max, e


def equilibrium_instance(p, drive, n_samples, settle, n_harm, offset=(0, 0, 0)):
    """Equilibrium model (model M0 of the data-driven models section, Eq. Langevin): the moment follows
    the field without delay and without anisotropy, m(t) = L(beta |H(t)|) H(t) / |H(t)| with
    L(x) = coth(x) - 1/x, dimensionless like the FP moment; sampled at the same times as
    solve_instance (the settling periods change nothing: the model has no memory) and reduced to the
    same harmonics.  Returns dict with m [N_s, 3] and Phi [n_harm+1, 3]."""
    sc = particle_scalars(p["D"], p["Ms"], p["K"], p["alpha"], p["T"])
    T = drive["period"]
    ts = settle * T + np.arange(n_samples) * T / n_samples
    B = drive_field(drive, offset, ts)                     # [N_s, 3], mu0 H in T
    bn = np.linalg.norm(B, axis=1)
    x = sc["beta_T"] * bn
    safe = np.where(bn > 0, bn, 1.0)
    m = np.where(bn[:, None] > 0, (langevin(x) / safe)[:, None] * B, 0.0)
    return dict(m=m, Phi=harmonics_from_samples(m, T, n_harm))


def boltzmann_mean(bH, sigma, n, nq=80):
    """<m> under f ~ exp(bH . m + sigma (n.m)^2) by product quadrature (bH = beta * H vector)."""
    th, ph, W = quadrature(nq, 2 * nq)
    mv, _, _ = unit_vectors(th, ph)
    e = mv @ np.asarray(bH, float) + sigma * (mv @ np.asarray(n, float)) ** 2
    w = W * np.exp(e - e.max())
    return (mv * w[:, None]).sum(0) / w.sum()


def azimuth_generator(L):
    """Matrix D_ij = int Y_i d/dphi Y_j (rotation about z) by quadrature; used by the rotating-field pin."""
    th, ph, W = quadrature(L + 6, 2 * L + 12)
    Y, G = real_sh(L, th, ph)
    mv, _, _ = unit_vectors(th, ph)
    zxm = np.cross(np.array([0.0, 0.0, 1.0])[None, :], mv)
    dphi = np.einsum("jqa,qa->jq", G, zxm)
    return (Y * W) @ dphi.T
