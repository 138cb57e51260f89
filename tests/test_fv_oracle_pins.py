"""Pins of the finite-volume cross-check (oracle/fv_oracle.py) and, through it, of the Galerkin oracle.

The finite-volume discretisation shares no algebra with the spherical-harmonic Galerkin oracle: it
takes the drift straight from Eq. convection (the p1..p4 terms), not from the reduced form the
Galerkin assembly uses.  Its pieces are pinned against geometry, closed forms and quadrature; the
whole is then pinned to the Galerkin oracle's dynamic solution, which it must approach at second
order in the mesh width, and a precession term of the wrong sign in the Galerkin oracle would sit
several times further away than the finite-volume error (shown below by flipping it).
"""
import numpy as np
import pytest

import oracle as O
import oracle.fp_oracle as FP
from oracle import fv_oracle as FV

MS, TB = 474e3, 295.0


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def meshes():
    return {k: FV.fv_mesh(k) for k in (1, 2, 3, 4)}


# ------------------------------------------------------------------ mesh ---

@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts_and_orientation(level):
    V, F = FV.icosphere(level)
    assert F.shape[0] == 20 * 4 ** level and V.shape[0] == 10 * 4 ** level + 2
    edges = {tuple(sorted((int(f[k]), int(f[(k + 1) % 3])))) for f in F for k in range(3)}
    assert len(edges) == 30 * 4 ** level
    assert V.shape[0] - len(edges) + F.shape[0] == 2                     # Euler characteristic
    np.testing.assert_allclose(np.linalg.norm(V, axis=1), 1.0, atol=1e-15)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    assert np.all(np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0)


def test_cell_geometry(meshes):
    for m in meshes.values():
        assert abs(m["area"].sum() - 4 * np.pi) < 1e-12                 # the sphere's area
        assert np.abs(m["mom"].sum(0)).max() < 1e-12                     # integral of m over the sphere
        # each directed edge has its twin, with the cells swapped
        twin = {(int(i), int(a), int(b)) for i, a, b in zip(m["cell"], m["P"], m["Q"])}
        assert all((int(j), int(b), int(a)) in twin for j, a, b in zip(m["nb"], m["P"], m["Q"]))
        assert np.all(m["nb"] != m["cell"])
        # the circumcentres of both cells are equidistant from the edge's end points
        for c in (m["centre"][m["cell"]], m["centre"][m["nb"]]):
            d = np.einsum("ij,ij->i", c, m["V"][m["P"]] - m["V"][m["Q"]])
            assert np.abs(d).max() < 1e-14
        # the cell centre is inside its triangle (the refined icosahedron's triangles are acute)
        V, F = m["V"], m["F"]
        for k in range(3):
            p, q = V[F[:, k]], V[F[:, (k + 1) % 3]]
            assert np.all(np.einsum("ij,ij->i", np.cross(p, q), m["centre"]) > 0)


def _subdivided_moment(a, b, c, depth):
    """Integral of m over the spherical triangle (a, b, c) by midpoint refinement (area x centroid)."""
    tris = [(a, b, c)]
    for _ in range(depth):
        nxt = []
        for p, q, r in tris:
            pq, qr, rp = (FV._unit(p + q), FV._unit(q + r), FV._unit(r + p))
            nxt += [(p, pq, rp), (pq, q, qr), (rp, qr, r), (pq, qr, rp)]
        tris = nxt
    P, Q, R = (np.array(x) for x in zip(*tris))
    trip = np.einsum("ij,ij->i", P, np.cross(Q, R))
    den = 1 + np.einsum("ij,ij->i", P, Q) + np.einsum("ij,ij->i", Q, R) + np.einsum("ij,ij->i", R, P)
    A = 2 * np.arctan2(np.abs(trip), den)
    return (A[:, None] * FV._unit(P + Q + R)).sum(0), A.sum()


def test_cell_moment_and_area_by_refinement(meshes):
    m = meshes[1]
    for cell in (0, 17, 55):
        a, b, c = m["V"][m["F"][cell]]
        mom5, _ = _subdivided_moment(a, b, c, 5)
        mom6, area = _subdivided_moment(a, b, c, 6)
        assert abs(area - m["area"][cell]) < 1e-13
        mom = (4 * mom6 - mom5) / 3              # the area x centroid rule is second order
        np.testing.assert_allclose(m["mom"][cell], mom, rtol=0, atol=1e-9 * m["area"][cell])


# ---------------------------------------------------------------- fluxes ---

def test_precession_edge_flux_is_the_line_integral_of_eq_convection(meshes):
    """psi(Q) - psi(P) equals the Gauss-Legendre line integral of (p1 H x m + p3 (n.m) n x m) . nu
    along the edge, nu the normal pointing out of the cell on the left of P -> Q."""
    m = meshes[2]
    sc = O.particle_scalars(20e-9, MS, 3e3, 0.1, TB)
    r = np.random.default_rng(5)
    n = FV._unit(r.normal(size=3))
    B = np.array([4e-3, -7e-3, 2e-3])
    H = B / O.MU0
    _, psi = FV.fv_potentials(sc, 0.1, n, B, m["V"])
    x, w = np.polynomial.legendre.leggauss(24)
    for e in r.choice(m["P"].size, 12, replace=False):
        P, Q = m["V"][m["P"][e]], m["V"][m["Q"][e]]
        th = m["ell"][e]
        s = 0.5 * th * (x + 1.0)
        pts = (np.sin(th - s)[:, None] * P + np.sin(s)[:, None] * Q) / np.sin(th)
        tang = (-np.cos(th - s)[:, None] * P + np.cos(s)[:, None] * Q) / np.sin(th)
        nu = np.cross(tang, pts)
        # nu points away from the cell's centre
        assert np.einsum("ij,j->i", nu, m["centre"][m["cell"][e]]).max() < 0
        b = sc["p1"] * np.cross(H, pts) + sc["p3"] * (pts @ n)[:, None] * np.cross(n, pts)
        flux = 0.5 * th * np.sum(w * np.einsum("ij,ij->i", b, nu))
        g = psi[m["Q"][e]] - psi[m["P"][e]]
        assert abs(flux - g) < 1e-11 * max(abs(g), sc["p1"] * np.linalg.norm(H) * th)


def test_bernoulli_function():
    x = np.array([-30.0, -1.0, -1e-6, 0.0, 3e-7, 0.5, 40.0])
    ref = np.array([1.0 if v == 0 else v / np.expm1(v) for v in x])
    np.testing.assert_allclose(FV.bernoulli(x), ref, rtol=1e-12)
    np.testing.assert_allclose(FV.bernoulli(x) - FV.bernoulli(-x), -x, rtol=1e-12, atol=1e-15)


def test_operator_conserves_probability_and_keeps_the_boltzmann_state(meshes):
    m = meshes[3]
    sc = O.particle_scalars(21e-9, MS, 4e3, 0.07, TB)
    n = FV._unit(np.array([0.3, -0.5, 0.8]))
    B = np.array([5e-3, 2e-3, -6e-3])
    K = FV.fv_operator(m, sc, 0.07, n, B)
    assert np.abs(np.asarray(K.sum(0))).max() < 1e-9 * np.abs(K).max()      # columns sum to zero
    fb = FV.boltzmann(m, sc, 0.07, n, B)
    Kg = FV.fv_operator(m, sc, 0.07, n, B, precession=0.0)
    assert np.abs(Kg @ fb).max() < 1e-10 * np.abs(Kg).max() * fb.max()       # exact for the gradient part
    # with precession the discrete null vector approaches the Boltzmann density as the mesh is refined
    errs = []
    for lev in (2, 3, 4):
        mm = meshes[lev]
        K = FV.fv_operator(mm, sc, 0.07, n, B).toarray()
        K[0, :] = mm["area"]
        rhs = np.zeros(K.shape[0])
        rhs[0] = 1.0
        f0 = np.linalg.solve(K, rhs)
        errs.append(rel(FV.fv_moment(mm, f0), FV.fv_moment(mm, FV.boltzmann(mm, sc, 0.07, n, B))))
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3 and errs[2] < 1e-3


# ---------------------------------------------------------- closed forms ---

def test_equilibrium_converges_to_langevin_at_second_order(meshes):
    sc = O.particle_scalars(20e-9, MS, 0.0, 0.1, TB)
    B = np.array([0.0, 0.0, 3e-3])
    x = sc["beta_T"] * 3e-3
    errs = [abs(FV.fv_moment(meshes[k], FV.boltzmann(meshes[k], sc, 0.1, [1, 0, 0], B))[2] - O.langevin(x))
            for k in (2, 3, 4)]
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_anisotropic_equilibrium_matches_quadrature(meshes):
    sc = O.particle_scalars(22e-9, MS, 3e3, 0.1, TB)
    n = FV._unit(np.array([1.0, 1.0, 0.5]))
    B = np.array([2e-3, -1e-3, 1e-3])
    ref = O.boltzmann_mean(sc["beta_T"] * B, sc["sigma"], n, nq=120)
    errs = [rel(FV.fv_moment(meshes[k], FV.boltzmann(meshes[k], sc, 0.1, n, B)), ref) for k in (3, 4)]
    assert errs[1] < errs[0] / 3 and errs[1] < 2e-3


def test_free_relaxation_rates_are_l_l_plus_1_over_2_tau(meshes):
    """Without field and anisotropy the density relaxes by diffusion alone: degree l decays at
    l (l + 1) / (2 tau), so the slowest rates are 1/tau (three-fold) and 3/tau (five-fold)."""
    sc = O.particle_scalars(20e-9, MS, 0.0, 0.1, TB)
    errs = []
    for k in (2, 3):
        m = meshes[k]
        A = FV.fv_operator(m, sc, 0.1, [0, 0, 1], np.zeros(3)).toarray() / m["area"][:, None]
        ev = np.sort(np.linalg.eigvals(A).real)[::-1][:9] * sc["tau"]
        assert abs(ev[0]) < 1e-9
        errs.append(np.abs(ev[1:4] + 1.0).max())
        np.testing.assert_allclose(ev[4:9], -3.0, rtol=2e-2)
    assert errs[0] / errs[1] > 3.5 and errs[1] < 2e-3


# ------------------------------------------------------------- dynamics ---

def _fast_case():
    """A fast drive (period 2 us, 1.5 / 2 / 0.5 MHz components), a tilted easy axis and weak damping,
    where the precession's sign moves <m> by about 2 %."""
    p = dict(D=18e-9, Ms=MS, K=2e3, alpha=0.05, T=TB)
    th = np.deg2rad(60.0)
    n = np.array([np.cos(th), 0.0, np.sin(th)])
    T = 2e-6
    drive = dict(amp=(10e-3, 8e-3, 3e-3), freq=(3 / T, 4 / T, 1 / T), phase=(0.0, 0.3, -0.7), period=T)
    return p, n, drive, (1e-3, -2e-3, 0.5e-3)


def test_bdf2_is_second_order_in_time(meshes):
    """BDF2's global error falls as h^2.  The precession term is switched off: its mesh-scale modes
    are stiff and oscillatory, and where |h lambda| crosses 1 for some of them the observed order
    wanders; the gradient part alone shows the integrator's order cleanly."""
    p = dict(D=20e-9, Ms=MS, K=2e3, alpha=0.1, T=TB)
    n = np.array([0.6, 0.0, 0.8])
    T = 40e-6
    drive = dict(amp=(10e-3, 8e-3, 3e-3), freq=(3 / T, 4 / T, 1 / T), phase=(0.0, 0.3, -0.7), period=T)
    ms = [FV.fv_solve_instance(p, n, 1, drive, 16, 1, r=r, offset=(1e-3, -2e-3, 5e-4), mesh=meshes[1],
                               precession=0.0)["m"] for r in (16, 32, 128)]
    e1, e2 = rel(ms[0], ms[2]), rel(ms[1], ms[2])
    # second order: errors against the finest run scale as (1 - 1/16) : (1/4 - 1/16) = 5
    # (first order would give 2.3)
    assert 4.0 < e1 / e2 < 6.5


def test_dynamics_conserve_probability(meshes):
    p, n, drive, off = _fast_case()
    res = FV.fv_solve_instance(p, n, 2, drive, 16, 1, r=4, offset=off, mesh=meshes[2])
    assert abs(res["mass"] - 1.0) < 1e-10
    assert np.all(np.linalg.norm(res["m"], axis=1) < 1.0)


def _flipped_components(L, n):
    c = dict(_ORIG_COMPONENTS(L, n))
    c["Fp"] = [-x for x in c["Fp"]]
    c["Gp"] = -c["Gp"]
    return c


_ORIG_COMPONENTS = FP.galerkin_components


def test_finite_volumes_converge_to_the_galerkin_oracle(meshes, monkeypatch):
    """The two discretisations of Eq. FP-general agree to the finite-volume error, which falls at
    second order; the Galerkin solution with the precession term's sign flipped is far outside."""
    p, n, drive, off = _fast_case()
    g = O.solve_instance(p, n, 14, drive, 64, 1, 8, r=4, offset=off)["m"]
    f2 = FV.fv_solve_instance(p, n, 2, drive, 64, 1, r=8, offset=off, mesh=meshes[2])["m"]
    f3 = FV.fv_solve_instance(p, n, 3, drive, 64, 1, r=8, offset=off, mesh=meshes[3])["m"]
    e2, e3 = rel(f2, g), rel(f3, g)
    assert e2 / e3 > 3.0 and e3 < 4e-3
    monkeypatch.setattr(FP, "galerkin_components", _flipped_components)
    gf = O.solve_instance(p, n, 14, drive, 64, 1, 8, r=4, offset=off)["m"]
    assert rel(f3, gf) > 4 * e3


# ------------------------------------------------- stored cross-check set ---

def _fv_goldens():
    import glob
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    return sorted(glob.glob(os.path.join(here, "fv_*.npz")))


@pytest.mark.parametrize("path", _fv_goldens())
def test_stored_finite_volume_solutions_pin_the_galerkin_oracle(path):
    """tests/golden/fv_*.npz (written by tests/golden/make_golden.py from oracle/ only): the
    finite-volume solutions on 1280, 5120 and 20480 triangles converge at second order, and their
    extrapolation agrees with the Galerkin oracle at degree L + 6 to within its own error; the
    Galerkin oracle at degree 4 is far outside, so the cross-check resolves truncation."""
    z = np.load(path)
    g = z["gal_L6"]
    e3, e4, e5 = (rel(z[k], g) for k in ("fv3", "fv4", "fv5"))
    assert e3 / e4 > 3.0 and e4 / e5 > 3.0
    R45 = (4 * z["fv5"] - z["fv4"]) / 3
    R34 = (4 * z["fv4"] - z["fv3"]) / 3
    err = rel(R45, R34) + rel(z["fv4"], z["fv4_half_r"]) / 3
    assert rel(g, R45) <= 2.0 * err + 1e-5
    assert rel(z["gal_4"], R45) > 10.0 * (2.0 * err + 1e-5)


@pytest.mark.parametrize("path", _fv_goldens())
def test_truncation_estimate_bounds_the_truncation_error(path):
    """The oracle's truncation estimate (stationary moments of degrees L and L - 2 under the largest
    sampled field) lies above the degree-L error of the periodic m(t) measured against the
    finite-volume reference, within a factor 30."""
    import workloads as W
    z = np.load(path)
    i = int(z["idx"])
    ws = W.fv_crosscheck()
    inst = {k: v[i] for k, v in ws["inst"].items()}
    p = dict(D=inst["D"], Ms=inst["Ms"], K=inst["K"], alpha=inst["alpha"], T=inst["T"])
    est = O.truncation_estimate(p, inst["easy_axis"], int(inst["L"]), ws["drive"], inst["offset"], ws["samples"])
    R45 = (4 * z["fv5"] - z["fv4"]) / 3
    R34 = (4 * z["fv4"] - z["fv3"]) / 3
    err = rel(R45, R34) + rel(z["fv4"], z["fv4_half_r"]) / 3
    trunc = rel(z["gal_L"], R45)
    assert est >= trunc - 2.0 * err
    assert est <= 30.0 * max(trunc, 2.0 * err)


def test_peak_field_picks_the_first_of_equal_maxima():
    T = 1e-5
    drive = dict(amp=(1e-2, 1e-2, 0.0), freq=(2 / T, 3 / T, 0.0), phase=(0.0, 0.0, 0.0), period=T)
    # at t = 0 both components are at +10 mT; at t = T/2 x is at +10 mT and y at -10 mT: a tie
    np.testing.assert_allclose(O.peak_field(drive, (0, 0, 0), 64), [1e-2, 1e-2, 0.0])
    # an offset in -y makes the second maximum the larger one
    np.testing.assert_allclose(O.peak_field(drive, (0, -1e-3, 0), 64), [1e-2, -1.1e-2, 0.0])
