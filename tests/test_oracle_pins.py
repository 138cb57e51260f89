"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test pins the oracle to something other than itself: a closed form, an
invariant, a library routine or brute force.  A plausible slip (a dropped term,
a wrong sign or index, a transposed operand) in the oracle fails at least one.
"""
import numpy as np
import pytest

import oracle as O

P_CFG1 = dict(D=20e-9, Ms=474e3, K=2e3, alpha=0.1, T=295.0)


def rng(seed):
    return np.random.default_rng(seed)


def random_unit(r):
    v = r.normal(size=3)
    return v / np.linalg.norm(v)


def random_rotation(r):
    q, _ = np.linalg.qr(r.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


# ------------------------------------------------------- particle scalars ---

def _half_unit(printed):
    """Half a unit in the last digit of a value printed as text."""
    dec = printed.split(".")[1] if "." in printed else ""
    return 0.5 * 10.0 ** (-len(dec))


@pytest.mark.parametrize("D,K,alpha,tau_ns,beta12,sigma", [
    (20e-9, 2e3, 0.1, "13.98", "5.85", "2.06"),      # the single-instance particle (magnetite, 295 K)
    (30e-9, 2e4, 0.05, "93.7", "19.7", "69.4"),      # the uneven sweep's stiffest corner
    (15e-9, 5e2, 0.3, "2.12", "2.47", "0.22"),       # ... and its softest corner
])
def test_particle_scalars_match_hand_computed_values(D, K, alpha, tau_ns, beta12, sigma):
    """tau (the constant after Eq. convection), beta * (12 mT / mu0) and sigma = K V_C / (k_B T) (model M0)
    against values worked out by hand from the definitions, independently of this code, to the digits
    shown (M_S = 474 kA/m, T = 295 K), within half a unit of the last digit.  They fix the absolute time
    scale that every other pin reads from the same function: a dropped factor 2, (1 + alpha^2), 1 / alpha
    or a radius for a diameter moves one of them by more than that; the three points tell the alpha
    dependence apart."""
    sc = O.particle_scalars(D, 474e3, K, alpha, 295.0)
    for got, want in ((sc["tau"] * 1e9, tau_ns), (sc["beta_T"] * 12e-3, beta12), (sc["sigma"], sigma)):
        assert abs(got - float(want)) <= _half_unit(want), (got, want)


# ---------------------------------------------------------------- basis ---

@pytest.mark.parametrize("L", [4, 10, 16])
def test_basis_orthonormal_and_convention(L):
    th, ph, W = O.quadrature(L + 6, 2 * L + 12)
    Y, G = O.real_sh(L, th, ph)
    N = (L + 1) ** 2
    assert np.abs((Y * W) @ Y.T - np.eye(N)).max() < 1e-12
    m, _, _ = O.unit_vectors(th, ph)
    c = np.sqrt(3 / (4 * np.pi))
    # no Condon-Shortley phase: Y_{1,1} ~ x, Y_{1,-1} ~ y, Y_{1,0} ~ z
    assert np.abs(Y[O.sh_index(1, 1)] - c * m[:, 0]).max() < 1e-14
    assert np.abs(Y[O.sh_index(1, -1)] - c * m[:, 1]).max() < 1e-14
    assert np.abs(Y[O.sh_index(1, 0)] - c * m[:, 2]).max() < 1e-14


@pytest.mark.parametrize("L", [6, 16])
def test_surface_gradient_stiffness_is_laplace_spectrum(L):
    """int grad Y_i . grad Y_j = l(l+1) delta_ij pins every gradient (theta and phi parts)."""
    th, ph, W = O.quadrature(L + 6, 2 * L + 12)
    Y, G = O.real_sh(L, th, ph)
    K = np.einsum("iqa,jqa,q->ij", G, G, W)
    ls = O.sh_degrees(L)
    assert np.abs(K - np.diag(ls * (ls + 1.0))).max() < 1e-9
    # gradients are tangent
    m, _, _ = O.unit_vectors(th, ph)
    assert np.abs(np.einsum("iqa,qa->iq", G, m)).max() < 1e-12


def test_quadrature_exactness_brute_force():
    """Product rule vs. brute-force closed-form moments of monomials on the sphere."""
    from math import gamma
    th, ph, W = O.quadrature(8, 16)
    m, _, _ = O.unit_vectors(th, ph)
    for (a, b, c) in [(0, 0, 0), (2, 0, 0), (2, 2, 0), (4, 2, 2), (6, 0, 4), (2, 2, 2)]:
        num = np.sum(W * m[:, 0] ** a * m[:, 1] ** b * m[:, 2] ** c)
        be = [(k + 1) / 2 for k in (a, b, c)]
        exact = 2 * gamma(be[0]) * gamma(be[1]) * gamma(be[2]) / gamma(sum(be))
        assert abs(num - exact) < 1e-13


# ------------------------------------------------------------ operator ---

def test_reduced_drift_equals_paper_drift():
    """2 tau b(m,H,n) with the paper's p1..p4 equals grad Phi - m x grad Phi / alpha (tangent form)."""
    r = rng(1)
    for _ in range(5):
        p = dict(D=r.uniform(12e-9, 30e-9), Ms=r.uniform(3e5, 5e5), K=r.uniform(100, 2e4),
                 alpha=r.uniform(0.05, 0.5), T=r.uniform(250, 320))
        sc = O.particle_scalars(**p)
        n = random_unit(r)
        B = r.normal(size=3) * 0.01            # mu0 H in tesla
        H = B / O.MU0
        m = random_unit(r)
        b = (sc["p1"] * np.cross(H, m) + sc["p2"] * np.cross(np.cross(m, H), m)
             + sc["p3"] * (n @ m) * np.cross(n, m) + sc["p4"] * (n @ m) * np.cross(np.cross(m, n), m))
        gradPhi = sc["beta_T"] * (B - (B @ m) * m) + 2 * sc["sigma"] * (n @ m) * (n - (n @ m) * m)
        v = gradPhi - np.cross(m, gradPhi) / p["alpha"]
        assert np.allclose(2 * sc["tau"] * b, v, rtol=1e-12, atol=1e-12 * np.abs(v).max())


def test_conservation_row_zero():
    """Total probability is conserved: row 0 of every piece vanishes."""
    r = rng(2)
    A0, Aa, _ = O.operator_parts(P_CFG1, random_unit(r), 10)
    scale = np.abs(A0).max()
    assert np.abs(A0[0]).max() < 1e-13 * scale
    for A in Aa:
        assert np.abs(A[0]).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_boltzmann_stationary(seed):
    """Static field: the stationary Galerkin state reproduces the Boltzmann mean of exp(beta H.m + sigma (n.m)^2).

    This pins the precession terms too (they must cancel for the Boltzmann density)."""
    r = rng(seed)
    n = random_unit(r)
    B = random_unit(r) * r.uniform(2e-3, 6e-3)
    p = dict(P_CFG1)
    p["alpha"] = r.uniform(0.05, 0.3)
    A0, Aa, sc = O.operator_parts(p, n, 16)
    A = A0 + sum(B[a] * Aa[a] for a in range(3))
    m = O.moment(O.stationary(A))
    mb = O.boltzmann_mean(sc["beta_T"] * B, sc["sigma"], n)
    assert np.abs(m - mb).max() < 1e-9


def test_langevin_limit_isotropic():
    """K = 0: <m> . H_hat = coth(beta|H|) - 1/(beta|H|) (paper Eq. Langevin)."""
    r = rng(6)
    p = dict(P_CFG1, K=0.0)
    n = random_unit(r)
    for mag in [0.5e-3, 3e-3, 8e-3]:
        hhat = random_unit(r)
        B = mag * hhat
        A0, Aa, sc = O.operator_parts(p, n, 24)
        A = A0 + sum(B[a] * Aa[a] for a in range(3))
        m = O.moment(O.stationary(A))
        x = sc["beta_T"] * mag
        assert abs(m @ hhat - O.langevin(x)) < 1e-10
        assert np.linalg.norm(m - (m @ hhat) * hhat) < 1e-10


def test_stationary_matches_svd_null_vector():
    r = rng(7)
    A0, Aa, _ = O.operator_parts(P_CFG1, random_unit(r), 8)
    A = A0 + 3e-3 * Aa[0] - 1e-3 * Aa[2]
    c = O.stationary(A)
    _, s, vh = np.linalg.svd(A)
    v = vh[-1] / vh[-1][0] * c[0]
    assert s[-1] < 1e-8 * s[0]
    assert np.abs(v - c).max() < 1e-11


# ---------------------------------------------------------- dynamics ---

def test_isotropic_diffusion_decay():
    """H = 0, K = 0: each coefficient decays as exp(-l(l+1) t / (2 tau))."""
    L = 6
    p = dict(P_CFG1, K=0.0)
    A0, Aa, sc = O.operator_parts(p, [0, 0, 1], L)
    r = rng(8)
    c0 = r.normal(size=(L + 1) ** 2)
    tau = sc["tau"]
    period = 2 * tau
    ns = 8
    cs = O.integrate_samples(lambda t: A0, c0, period, ns, 0, 32)
    ls = O.sh_degrees(L)
    ts = np.arange(ns) * period / ns
    exact = c0[None, :] * np.exp(-ls[None, :] * (ls[None, :] + 1) * ts[:, None] / (2 * tau))
    assert np.abs(cs - exact).max() < 1e-7 * np.abs(c0).max()


def test_radau_order_five():
    """y' = cos(t) y, y(0) = 1 has y = exp(sin t); global error falls as h^5."""
    errs = []
    for r in [2, 4, 8]:
        cs = O.integrate_samples(lambda t: np.array([[np.cos(t)]]), [1.0], 2.0, 2, 0, r)
        errs.append(abs(cs[1, 0] - np.exp(np.sin(1.0))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.6), orders


def test_probability_conserved_in_time():
    r = rng(9)
    drive = dict(amp=(12e-3, 0, 0), freq=(25e3, 0, 0), phase=(0, 0, 0), period=40e-6)
    res = O.solve_instance(P_CFG1, random_unit(r), 8, drive, 40, 0, 5, r=1)
    assert abs(res["c_last"][0] - 1 / np.sqrt(4 * np.pi)) < 1e-15


def test_debye_linear_response():
    """K = 0, weak drive beta*H0 = 1e-3: bin 1 of m_x equals (beta H0 / 6) / (1 + i omega tau)."""
    p = dict(P_CFG1, K=0.0)
    sc = O.particle_scalars(**p)
    H0 = 1e-3 / sc["beta_T"]
    f = 5e6
    drive = dict(amp=(H0, 0, 0), freq=(f, 0, 0), phase=(0, 0, 0), period=1 / f)
    ns = 32
    res = O.solve_instance(p, [0, 0, 1], 4, drive, ns, 6, 2, r=4)
    M1 = np.sum(res["m"][:, 0] * np.exp(-2j * np.pi * np.arange(ns) / ns)) / ns
    omega_tau = 2 * np.pi * f * sc["tau"]
    pred = (1e-3 / 6) / (1 + 1j * omega_tau)
    assert abs(M1 - pred) < 2e-5 * abs(pred)
    assert abs(res["Phi"][1, 0] - (2j * np.pi * f) * pred) < 2e-5 * abs(2j * np.pi * f * pred)


def test_rotating_field_matches_rotating_frame_null_vector():
    """n = z, H = H0 (cos wt, sin wt, 0): settled m(t) = R_z(wt) m_rot, with m_rot from the
    null vector of the static rotating-frame operator A(H0 x) + w d/dphi."""
    L = 10
    f = 25e3
    H0 = 8e-3
    drive = dict(amp=(H0, H0, 0), freq=(f, f, 0), phase=(0, -np.pi / 2, 0), period=1 / f)
    ns = 100
    res = O.solve_instance(P_CFG1, [0, 0, 1], L, drive, ns, 2, 3, r=2)
    A0, Aa, _ = O.operator_parts(P_CFG1, [0, 0, 1], L)
    g = O.stationary(A0 + H0 * Aa[0] + 2 * np.pi * f * O.azimuth_generator(L))
    mg = O.moment(g)
    w = 2 * np.pi * f
    ts = 2 / f + np.arange(ns) / (ns * f)
    pred = np.stack([np.cos(w * ts) * mg[0] - np.sin(w * ts) * mg[1],
                     np.sin(w * ts) * mg[0] + np.cos(w * ts) * mg[1],
                     np.full(ns, mg[2])], 1)
    assert np.abs(pred - res["m"]).max() < 1e-9


def test_rotation_invariance():
    """m(Qn, QH(t)) = Q m(n, H(t)) for a proper rotation Q (static and driven)."""
    r = rng(10)
    Q = random_rotation(r)
    n = random_unit(r)
    B = random_unit(r) * 5e-3
    L = 10
    A0, Aa, _ = O.operator_parts(P_CFG1, n, L)
    m1 = O.moment(O.stationary(A0 + sum(B[a] * Aa[a] for a in range(3))))
    A0q, Aaq, _ = O.operator_parts(P_CFG1, Q @ n, L)
    QB = Q @ B
    m2 = O.moment(O.stationary(A0q + sum(QB[a] * Aaq[a] for a in range(3))))
    assert np.abs(Q @ m1 - m2).max() < 1e-12
    # driven along a rotated 1D axis
    e = np.array([1.0, 0.0, 0.0])
    amp = 10e-3
    d1 = dict(amp=tuple(amp * e), freq=(25e3,) * 3, phase=(0, 0, 0), period=40e-6)
    d2 = dict(amp=tuple(amp * (Q @ e)), freq=(25e3,) * 3, phase=(0, 0, 0), period=40e-6)
    off = np.array([1e-3, -2e-3, 0.5e-3])
    ra = O.solve_instance(P_CFG1, n, 8, d1, 40, 1, 4, r=1, offset=off)
    rb = O.solve_instance(P_CFG1, Q @ n, 8, d2, 40, 1, 4, r=1, offset=Q @ off)
    assert np.abs(ra["m"] @ Q.T - rb["m"]).max() < 1e-11


def test_axisymmetric_drive_half_wave_symmetry():
    """K = 0, 1D drive along x, zero offset: m stays on x and even harmonics vanish."""
    p = dict(P_CFG1, K=0.0)
    drive = dict(amp=(12e-3, 0, 0), freq=(25e3, 0, 0), phase=(0, 0, 0), period=40e-6)
    res = O.solve_instance(p, [0.3, 0.4, np.sqrt(0.75)], 10, drive, 64, 2, 8, r=1)
    assert np.abs(res["m"][:, 1:]).max() < 1e-12
    ph = np.abs(res["Phi"][:, 0])
    assert ph[[0, 2, 4, 6, 8]].max() < 1e-9 * ph[1]


# ------------------------------------------------------------ signal ---

def test_harmonics_match_library_fft_and_band_limited_derivative():
    r = rng(11)
    T = 1e-3
    ns = 64
    m = r.normal(size=(ns, 3))
    Phi = O.harmonics_from_samples(m, T, 20)
    F = np.fft.fft(m, axis=0) / ns
    k = np.arange(21)
    assert np.abs(Phi - (2j * np.pi * k / T)[:, None] * F[:21]).max() < 1e-12 * np.abs(Phi).max()
    # band-limited: m = cos(2 pi 3 t / T) => Phi_3 = (2 pi i 3 / T) / 2, others 0
    t = np.arange(ns) * T / ns
    Phi = O.harmonics_from_samples(np.cos(2 * np.pi * 3 * t / T)[:, None], T, 10)
    assert abs(Phi[3, 0] - 1j * np.pi * 3 / T) < 1e-10 * (3 / T)
    assert np.abs(np.delete(Phi[:, 0], 3)).max() < 1e-10 * (3 / T)


def test_exact_by_parts_route_agrees_with_rhs_route_when_resolved():
    """When the trajectory is band-limited well below Nyquist (slow drive, weak field),
    the by-parts harmonics equal the rectangle rule on RHS-evaluated dm/dt."""
    p = dict(P_CFG1)
    drive = dict(amp=(2e-3, 1e-3, 0), freq=(25e3, 50e3, 0), phase=(0, 0, 0), period=40e-6)
    res = O.solve_instance(p, [np.cos(0.5), np.sin(0.5), 0], 8, drive, 400, 1, 10, r=2)
    a, b = res["Phi"][1:, :2], res["Phi_rect"][1:, :2]
    assert np.linalg.norm(a - b) < 1e-6 * np.linalg.norm(b)


# ------------------------------------------------- finite-difference derivatives ---
# The sensitivity references are central differences of the oracle; these pins check that the
# differencing recipe (step sizes, angle parametrisation) reproduces closed forms.

def _stationary_m(D, K, n, B, L=16):
    p = dict(D=D, Ms=474e3, K=K, alpha=0.1, T=295.0)
    A0, Aa, _ = O.operator_parts(p, n, L)
    return O.moment(O.stationary(A0 + sum(B[a] * Aa[a] for a in range(3))))


def test_central_difference_in_D_matches_langevin_derivative():
    """K = 0: m = L(x) H/|H| with x = beta |H| and beta proportional to D^3, so
    dm/dD = L'(x) (3 x / D) H/|H|, L'(x) = 1/x^2 - 1/sinh(x)^2."""
    B = np.array([4e-3, -2e-3, 3e-3])
    D = 18e-9
    n = np.array([0.0, 0.0, 1.0])
    h = 1e-6 * D
    fd = (_stationary_m(D + h, 0.0, n, B) - _stationary_m(D - h, 0.0, n, B)) / (2 * h)
    x = O.particle_scalars(D, 474e3, 0.0, 0.1, 295.0)["beta_T"] * np.linalg.norm(B)
    dL = 1 / x ** 2 - 1 / np.sinh(x) ** 2
    exact = dL * 3 * x / D * B / np.linalg.norm(B)
    assert np.abs(fd - exact).max() < 1e-6 * np.abs(exact).max()


def test_isotropic_particle_has_no_axis_angle_derivative():
    """K = 0 makes the easy axis irrelevant: central differences in both axis angles vanish."""
    ws_drive = dict(amp=(10e-3, 8e-3, 3e-3), freq=(3 / 40e-6, 4 / 40e-6, 1 / 40e-6), phase=(0.0, 0.3, -0.7),
                    period=40e-6)
    p = dict(D=18e-9, Ms=474e3, K=0.0, alpha=0.1, T=295.0)
    th, ph = 0.9, 0.4

    def phi(th, ph):
        n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        return O.solve_instance(p, n, 4, ws_drive, 16, 0, 4, r=2, offset=(1e-3, 0, 0))["Phi"]

    base = np.linalg.norm(phi(th, ph))
    for dth, dph in ((1e-6, 0.0), (0.0, 1e-6)):
        d = (phi(th + dth, ph + dph) - phi(th - dth, ph - dph)) / 2e-6
        assert np.linalg.norm(d) < 1e-6 * base


def test_equilibrium_model_is_the_isotropic_stationary_moment_of_each_instant():
    """Model M0 (Eq. Langevin): at every sample the equilibrium moment equals the stationary moment of
    the Fokker-Planck operator with K = 0 for the instantaneous field (an independent construction:
    Galerkin null vector at L = 24)."""
    p = dict(P_CFG1, D=14e-9, K=0.0)
    d = dict(amp=(12e-3, 12e-3, 0.0), freq=(2.5e6 / 102, 2.5e6 / 96, 0.0), phase=(0.0, 0.0, 0.0),
             period=652.8e-6)
    off = np.array([3e-3, -5e-3, 1e-3])
    eq = O.equilibrium_instance(p, d, 32, 1, 4, offset=off)
    A0, Aa, _ = O.operator_parts(p, np.array([0.0, 0.0, 1.0]), 24)
    for j in (0, 5, 11, 26):
        t = d["period"] * (1 + j / 32)
        B = O.drive_field(d, off, t)
        m = O.moment(O.stationary(A0 + sum(B[a] * Aa[a] for a in range(3))))
        assert np.abs(eq["m"][j] - m).max() < 1e-9


def test_equilibrium_model_symmetry_and_zero_field():
    """1D drive along x without offset: m stays on x and m(t + T/2) = -m(t), so the even harmonics
    vanish; at a zero field the moment is zero."""
    d = dict(amp=(12e-3, 0.0, 0.0), freq=(25e3, 0.0, 0.0), phase=(0.0, 0.0, 0.0), period=40e-6)
    eq = O.equilibrium_instance(P_CFG1, d, 64, 0, 10)
    assert np.abs(eq["m"][:, 1:]).max() == 0.0
    assert np.allclose(eq["m"][32:], -eq["m"][:32], rtol=0, atol=1e-13)
    scale = np.abs(eq["Phi"][1, 0])
    assert np.abs(eq["Phi"][0::2]).max() < 1e-12 * scale and np.abs(eq["Phi"][3, 0]) > 1e-3 * scale
    z = O.equilibrium_instance(P_CFG1, dict(d, amp=(0.0, 0.0, 0.0)), 8, 0, 2)
    assert np.array_equal(z["m"], np.zeros((8, 3)))
