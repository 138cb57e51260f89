"""Finite-volume cross-check of the Fokker-Planck model (TEST INFRASTRUCTURE, plain FP64).

This module is test infrastructure only, like the rest of ``oracle/``: it may be imported by
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` and shares no
code with the HIP library.

The paper solves Eq. FP-general with finite volumes: the sphere is cut into spherical triangles,
the probability flow over each edge gives one ODE per triangle, and a multistep integrator steps
the ODE system (Methods, "Particle magnetization model", the paragraph after Eq. convection).  This
is an independent discretisation of the same equation as the spherical-harmonic Galerkin oracle in
``fp_oracle`` and converges to the same solution as the mesh is refined; the tests use it to pin the
Galerkin oracle's dynamics (drift, precession sign, time scale) by a route that shares none of its
algebra.  The discrete definitions below (mesh, fluxes, integrator) are this project's readings;
the paper names none of them.

Mesh.  The icosahedron (its 20 faces from the convex hull of its 12 vertices, a library
primitive) refined ``level`` times: each spherical triangle is split into four by its edge
midpoints pushed out to the sphere.  Cells are the triangles (20 * 4**level), oriented
counter-clockwise seen from outside.  Per cell: exact spherical area (spherical excess), the
circumcentre on the sphere as the cell centre (the great circle joining two neighbouring
circumcentres crosses their common edge at a right angle, which makes the two-point flux below
consistent), and the exact cell integral of the unit vector m (half the sum over the edges of the
edge angle times the unit normal of the edge's great-circle plane).

Fluxes.  Eq. convection splits into a gradient part and a precession part:
  p2 (m x H) x m + p4 (n.m)(m x n) x m = grad_S U,   U   = p2 H.m + (p4/2) (n.m)^2,
  p1 H x m + p3 (n.m) n x m           = -m x grad psi, psi = p1 H.m + (p3/2) (n.m)^2.
With D = 1/(2 tau) the gradient part and the diffusion form D (f grad Phi - grad f), Phi = U / D,
whose flux from cell i to neighbour j over an edge of length l_ij is taken with the exponentially
fitted (Scharfetter-Gummel) two-point formula
  F_ij = D l_ij / d_ij * [ B(-(Phi_j - Phi_i)) f_i - B(Phi_j - Phi_i) f_j ],  B(x) = x / (e^x - 1),
d_ij the arc between the two centres, Phi taken at the centres; it vanishes exactly on the discrete
Boltzmann density f_i ~ exp(Phi_i).  The precession field -m x grad psi is divergence-free on the
sphere and its flux through an edge traversed from P to Q with the cell on the left is exactly
psi(Q) - psi(P); it carries the face value (f_i + f_j) / 2.  Cell balance:
  A_i df_i/dt = - sum over the three edges of (F_ij + (psi(Q) - psi(P)) (f_i + f_j) / 2),
so sum_i A_i f_i is conserved exactly (every flux leaves one cell and enters another).

Integrator.  BDF2 with a fixed step h = T / (N_s r) (one implicit Euler step to start), each step a
sparse direct solve (a library primitive); the operator is assembled at the new time.  Initial
state: the discrete Boltzmann density of the field at t = 0 with sum_i A_i f_i = 1; the samples are
those of (settle + 1) periods, the last one recorded, as in ``fp_oracle.integrate_samples``.

Mean moment (Eq. mean_magmom_FP / m0): sum_i f_i * (cell integral of m).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.spatial import ConvexHull

from .fp_oracle import particle_scalars, drive_field, harmonics_from_samples, MU0


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def icosphere(level):
    """Vertices [nv, 3] and counter-clockwise (outward) triangles [nf, 3] of the refined icosahedron."""
    g = (1.0 + np.sqrt(5.0)) / 2.0
    base = []
    for a in (-1.0, 1.0):
        for b in (-g, g):
            base += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    V = _unit(np.array(base))
    F = ConvexHull(V).simplices.copy()
    V, F = list(V), [tuple(int(x) for x in f) for f in F]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                mid[key] = len(V)
                V.append(_unit(V[a] + V[b]))
            return mid[key]

        out = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            out += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        F = out
    V = np.array(V)
    F = np.array(F, dtype=np.int64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def arc(p, q):
    """Great-circle angle between unit vectors (rows)."""
    return np.arctan2(np.linalg.norm(np.cross(p, q), axis=-1), np.einsum("ij,ij->i", p, q))


def fv_mesh(level):
    """Cells, their geometry and the list of interior edges (each once per side).

    Returns dict with V, F, area [nf], centre [nf, 3] (circumcentre), mom [nf, 3] (integral of m over
    the cell), and per directed edge arrays (3 nf of them, edge k of cell i runs from F[i, k] to
    F[i, k+1 mod 3]): cell, nb (the neighbour across it), P, Q (vertex indices), ell (arc length),
    dist (arc between the two centres).
    """
    V, F = icosphere(level)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    triple = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + np.einsum("ij,ij->i", c, a)
    area = 2.0 * np.arctan2(np.abs(triple), den)
    centre = _unit(np.cross(b - a, c - a))
    nf = F.shape[0]
    cell = np.repeat(np.arange(nf), 3)
    P = F.reshape(-1)
    Q = F[:, [1, 2, 0]].reshape(-1)
    owner = {(int(p), int(q)): int(i) for p, q, i in zip(P, Q, cell)}
    nb = np.array([owner[(int(q), int(p))] for p, q in zip(P, Q)], dtype=np.int64)
    ell = arc(V[P], V[Q])
    dist = arc(centre[cell], centre[nb])
    nrm = _unit(np.cross(V[P], V[Q]))
    mom = 0.5 * np.add.reduceat((ell[:, None] * nrm), np.arange(0, 3 * nf, 3), axis=0)
    return dict(V=V, F=F, area=area, centre=centre, mom=mom, cell=cell, nb=nb, P=P, Q=Q, ell=ell,
                dist=dist, level=level)


def bernoulli(x):
    """B(x) = x / (e^x - 1), B(0) = 1 (series below |x| < 1e-5)."""
    x = np.asarray(x, float)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-5
    xs = x[small]
    out[small] = 1.0 - xs / 2.0 + xs * xs / 12.0
    xl = x[~small]
    out[~small] = xl / np.expm1(xl)
    return out


def fv_potentials(sc, alpha, n, B, pts):
    """(Phi, psi) at unit vectors ``pts`` for mu0 H = B [T], from the constants of Eq. convection."""
    H = np.asarray(B, float) / MU0
    nm = pts @ np.asarray(n, float)
    Hm = pts @ H
    U = sc["p2"] * Hm + 0.5 * sc["p4"] * nm ** 2
    psi = sc["p1"] * Hm + 0.5 * sc["p3"] * nm ** 2
    return 2.0 * sc["tau"] * U, psi


def fv_operator(mesh, sc, alpha, n, B, precession=1.0):
    """Sparse K with A_i df_i/dt = (K f)_i at field mu0 H = B (columns sum to zero).

    ``precession`` scales the precession fluxes (1 = Eq. convection; the tests use 0 and -1 to show
    that the cross-checks see the term and its sign)."""
    D = 1.0 / (2.0 * sc["tau"])
    Phi_c, _ = fv_potentials(sc, alpha, n, B, mesh["centre"])
    _, psi_v = fv_potentials(sc, alpha, n, B, mesh["V"])
    i, j = mesh["cell"], mesh["nb"]
    w = D * mesh["ell"] / mesh["dist"]
    dPhi = Phi_c[j] - Phi_c[i]
    g = precession * (psi_v[mesh["Q"]] - psi_v[mesh["P"]])
    # outflow of cell i over this edge = cii * f_i + cij * f_j
    cii = w * bernoulli(-dPhi) + 0.5 * g
    cij = -w * bernoulli(dPhi) + 0.5 * g
    nf = mesh["area"].size
    K = sp.coo_matrix((np.concatenate([-cii, -cij]), (np.concatenate([i, i]), np.concatenate([i, j]))),
                      shape=(nf, nf)).tocsr()
    return K


def boltzmann(mesh, sc, alpha, n, B):
    """Discrete Boltzmann density f_i ~ exp(Phi(c_i)) with sum_i A_i f_i = 1."""
    Phi_c, _ = fv_potentials(sc, alpha, n, B, mesh["centre"])
    f = np.exp(Phi_c - Phi_c.max())
    return f / (mesh["area"] @ f)


def fv_moment(mesh, f):
    """<m> = sum_i f_i * integral of m over cell i (Eq. mean_magmom_FP / m0); f is [..., nf]."""
    return f @ mesh["mom"]


def fv_solve_instance(p, n, level, drive, n_samples, settle, r=2, offset=(0, 0, 0), n_harm=None,
                      mesh=None, precession=1.0):
    """Finite-volume solve of one instance: Boltzmann start at t = 0, BDF2 with r steps per sample.

    ``p`` holds D, Ms, K, alpha, T (SI units), ``n`` the easy axis.  Returns dict with m [N_s, 3]
    (lab frame, dimensionless), Phi (harmonics of dm/dt if n_harm is given), the final density and
    its total probability.
    """
    mesh = fv_mesh(level) if mesh is None else mesh
    sc = particle_scalars(p["D"], p["Ms"], p["K"], p["alpha"], p["T"])
    offset = np.asarray(offset, float)
    T = drive["period"]
    h = T / (n_samples * r)
    Adiag = sp.diags(mesh["area"])
    f = boltzmann(mesh, sc, p["alpha"], n, drive_field(drive, offset, 0.0))
    f_old = None
    out = np.zeros((n_samples, 3))
    first = settle * n_samples * r
    for step in range((settle + 1) * n_samples * r):
        if step >= first and (step - first) % r == 0:
            out[(step - first) // r] = fv_moment(mesh, f)
        K = fv_operator(mesh, sc, p["alpha"], n, drive_field(drive, offset, (step + 1) * h), precession)
        if f_old is None:
            M = (Adiag - h * K).tocsc()
            rhs = mesh["area"] * f
        else:
            M = (1.5 * Adiag - h * K).tocsc()
            rhs = mesh["area"] * (2.0 * f - 0.5 * f_old)
        f_old, f = f, spla.spsolve(M, rhs)
    res = dict(m=out, f=f, mass=float(mesh["area"] @ f), level=level, r=r, scalars=sc)
    if n_harm is not None:
        res["Phi"] = harmonics_from_samples(out, T, n_harm)
    return res
