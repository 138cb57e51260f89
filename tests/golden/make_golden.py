"""Write oracle reference outputs for the parity tests (calls only oracle/ and workloads/).

Each file holds, for one instance of a named workload: m [N_s, 3], Phi [K_h+1, 3]
(complex), the Radau refinement r used and the change against the run with r/2
(time-discretisation error estimate); the finite-volume cross-check files ("fv") hold the
finite-volume solutions on three meshes and Galerkin oracle solutions at three degrees.  Run:  python tests/golden/make_golden.py [names...]
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

def tangent_l10():
    return W.small_random(2, 10, seed=510, samples=48, settle=1, n_harm=8)


def wide_l17():
    return W.small_random(2, 17, seed=117, samples=48, settle=1, n_harm=8)


def wide_l20():
    return W.small_random(2, 20, seed=120, samples=48, settle=1, n_harm=8)


def wide_l24():
    return W.small_random(2, 24, seed=124, samples=48, settle=1, n_harm=8)


def identification_a0():
    """Angle 0 of the identification problem at the guess parameters, 64 harmonics (the first attempted
    step of these instances, one sample spacing long, overflows the FP32 factorisation)."""
    ws = W.identification_problem()
    out = W.identification_instances(ws, 0)
    out["n_harm"] = 64
    return out


def lissajous_stratified():
    """The 64 stratified instances of the Lissajous batch (workloads.lissajous_stratified_ids)."""
    return W.lissajous_stratified_ids()


UNEVEN_BUCKETS = ((8, 8), (9, 12), (13, 16), (17, 20), (21, 23), (24, 24))


def uneven_stratified():
    """Three resolvable instances of the 4096-instance uneven sweep per degree bucket (UNEVEN_BUCKETS):
    the band top (largest sigma - (L - 4), the stiffest particle its degree resolves by the rule), the
    instance with the median sigma of the bucket, and the one with the largest damping alpha (the
    truncated operator of a weakly damped particle is the least well resolved)."""
    ws = W.uneven_sweep(4096, seed=3)
    inst = ws["inst"]
    sig = W.anisotropy_ratio(inst["D"], inst["K"])
    ok = W.resolvable(inst["D"], inst["K"], inst["L"])
    ids = []
    for lo, hi in UNEVEN_BUCKETS:
        cand = np.nonzero(ok & (inst["L"] >= lo) & (inst["L"] <= hi))[0]
        top = cand[np.argmax(sig[cand] - (inst["L"][cand] - 4))]
        med = cand[np.argsort(sig[cand])[cand.size // 2]]
        damp = cand[np.argmax(inst["alpha"][cand])]
        ids += [int(top), int(med), int(damp)]
    return ids


def uneven_ws():
    return W.uneven_sweep(4096, seed=3)


# (workload factory, instance ids, Radau steps per sample for the reference and its check)
JOBS = {
    "tangent_l10": (tangent_l10, [0, 1], 8),
    "wide_l17": (wide_l17, [0], 8),
    "wide_l20": (wide_l20, [0, 1], 8),
    "wide_l24": (wide_l24, [0, 1], 16),
    "single_1d": (W.single_1d, [0], 8),
    # offset (3.5, 6.6) mT components 0 and 2, offset (12, 12) mT component 2
    "identification_a0": (identification_a0, [(24 * 32 + 20) * 4 + 0, (24 * 32 + 20) * 4 + 2, (31 * 32 + 31) * 4 + 2], 4),
    # finite differences at the production size (Radau IIA r = 4: with r = 2 the differences of these
    # stiff solves are off by up to 2.6e-4 relative, against the 1e-4 bound of the tangent tests)
    "tangent_ident": (identification_a0, [(24 * 32 + 20) * 4 + 0, (24 * 32 + 20) * 4 + 2], 4),
    "lissajous": (W.lissajous_grid, [(0 * 17 + 8) * 17 + 8, (3 * 17 + 2) * 17 + 13, (5 * 17 + 16) * 17 + 0,
                                     (7 * 17 + 10) * 17 + 4, (2 * 17 + 0) * 17 + 16, (6 * 17 + 12) * 17 + 12], 4),
    "lissajous_strat": (W.lissajous_grid, lissajous_stratified(), 4),
    "uneven": (uneven_ws, uneven_stratified(), 4),
    # finite-volume cross-check (BDF2 steps per sample)
    "fv": (W.fv_crosscheck, [0, 1, 2, 3, 4, 5], 32),
}


def _fd_solve(spec):
    """One oracle solve at perturbed parameters (D, K, alpha, polar and azimuth angle of the axis)."""
    factory, idx, r, D, K, alpha, th, ph = spec
    ws = factory()
    inst = {k: v[idx] for k, v in ws["inst"].items()}
    p = dict(D=D, Ms=inst["Ms"], K=K, alpha=alpha, T=inst["T"])
    ax = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    o = O.solve_instance(p, ax, int(inst["L"]), ws["drive"], ws["samples"], ws["settle"], ws["n_harm"], r=r,
                         offset=inst["offset"])
    return o["m"], o["Phi"]


def fd_one(args, pool=None):
    """Central finite differences of the oracle's m and Phi with respect to D, K, alpha and the
    easy-axis polar / azimuth angles (relative step 1e-6 for D, K, alpha; 1e-6 rad for the angles).
    The ten solves run in `pool` when one is given."""
    name, factory, idx, r = args
    ws = factory()
    inst = {k: v[idx] for k, v in ws["inst"].items()}
    n = np.asarray(inst["easy_axis"], float)
    th, ph = np.arccos(np.clip(n[2], -1, 1)), np.arctan2(n[1], n[0])
    t0 = time.time()
    base = [inst["D"], inst["K"], inst["alpha"], th, ph]
    steps = [1e-6 * inst["D"], 1e-6 * inst["K"], 1e-6 * inst["alpha"], 1e-6, 1e-6]
    specs = []
    for k in range(5):
        for sgn in (1, -1):
            v = list(base)
            v[k] += sgn * steps[k]
            specs.append((factory, idx, r, *v))
    res = list(pool.map(_fd_solve, specs)) if pool is not None else [_fd_solve(x) for x in specs]
    dm, dPhi = [], []
    for k in range(5):
        (ma, pa), (mb, pb) = res[2 * k], res[2 * k + 1]
        dm.append((ma - mb) / (2 * steps[k]))
        dPhi.append((pa - pb) / (2 * steps[k]))
    out = os.path.join(HERE, f"{name}_{idx}.npz")
    np.savez_compressed(out, dm=np.array(dm), dPhi=np.array(dPhi), r=r, idx=idx, theta=th, phi=ph)
    return f"{out}: finite differences of the oracle, r={r} ({time.time() - t0:.0f}s)"


def fv_one(args):
    """Finite-volume solutions of one instance on the refined icosahedron of levels 3, 4 and 5
    (1280, 5120 and 20480 triangles) with BDF2 at 32 steps per sample, level 4 also at 16 (time-error
    estimate), and the Galerkin oracle at the instance's degree L, at L + 6 and at L = 4 (a degree
    too low for these particles, to show the cross-check sees truncation)."""
    name, factory, idx, r = args
    from oracle import fv_oracle as FV
    ws = factory()
    inst = {k: v[idx] for k, v in ws["inst"].items()}
    p = dict(D=inst["D"], Ms=inst["Ms"], K=inst["K"], alpha=inst["alpha"], T=inst["T"])
    t0 = time.time()
    kw = dict(offset=inst["offset"])
    fv = {}
    for lev, rr in ((3, r), (4, r), (5, r), (4, r // 2)):
        fv[(lev, rr)] = FV.fv_solve_instance(p, inst["easy_axis"], lev, ws["drive"], ws["samples"], ws["settle"],
                                             r=rr, **kw)["m"]
    L = int(inst["L"])
    gal = {}
    for LL in (L, L + 6, 4):
        gal[LL] = O.solve_instance(p, inst["easy_axis"], LL, ws["drive"], ws["samples"], ws["settle"], ws["n_harm"],
                                   r=8, **kw)["m"]
    out = os.path.join(HERE, f"{name}_{idx}.npz")
    np.savez_compressed(out, fv3=fv[(3, r)], fv4=fv[(4, r)], fv5=fv[(5, r)], fv4_half_r=fv[(4, r // 2)], r=r,
                        gal_L=gal[L], gal_L6=gal[L + 6], gal_4=gal[4], L=L, idx=idx)
    R45 = (4 * fv[(5, r)] - fv[(4, r)]) / 3
    e = np.linalg.norm(gal[L] - R45) / np.linalg.norm(R45)
    return f"{out}: L={L} Galerkin vs extrapolated finite volumes {e:.2e} ({time.time() - t0:.0f}s)"


def one(args):
    name, factory, idx, r = args
    ws = factory()
    inst = {k: v[idx] for k, v in ws["inst"].items()}
    p = dict(D=inst["D"], Ms=inst["Ms"], K=inst["K"], alpha=inst["alpha"], T=inst["T"])
    t0 = time.time()
    kw = dict(offset=inst["offset"])
    fine = O.solve_instance(p, inst["easy_axis"], int(inst["L"]), ws["drive"], ws["samples"], ws["settle"],
                            ws["n_harm"], r=r, **kw)
    coarse = O.solve_instance(p, inst["easy_axis"], int(inst["L"]), ws["drive"], ws["samples"], ws["settle"],
                              ws["n_harm"], r=r // 2, **kw)
    err = np.linalg.norm(fine["Phi"] - coarse["Phi"]) / np.linalg.norm(fine["Phi"])
    out = os.path.join(HERE, f"{name}_{idx}.npz")
    np.savez_compressed(out, m=fine["m"], Phi=fine["Phi"], r=r, err_est=err, idx=idx,
                        Phi_rect=fine["Phi_rect"])
    return f"{out}: r={r} change vs r/2 = {err:.2e} ({time.time() - t0:.0f}s)"


if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    tasks = []
    for nm in names:
        nm, _, only = nm.partition(":")  # name:idx runs one instance of a job
        factory, ids, r = JOBS[nm]
        if nm == "uneven":
            # the cheap low degrees of the uneven sweep with twice the steps: at r = 4 the change against
            # r = 2 reaches 5e-6 there (fast drive-following particles), above the 2e-6 the tests require
            Ls = factory()["inst"]["L"]
            tasks += [(nm, factory, i, 8 if Ls[i] <= 13 else r) for i in ids if not only or i == int(only)]
        else:
            tasks += [(nm, factory, i, r) for i in ids if not only or i == int(only)]
    plain = [t for t in tasks if not t[0].startswith("tangent") and t[0] != "fv"]
    fvt = [t for t in tasks if t[0] == "fv"]
    if os.environ.get("GOLDEN_SKIP_EXISTING"):
        plain = [t for t in plain if not os.path.exists(os.path.join(HERE, f"{t[0]}_{t[2]}.npz"))]
    plain.sort(key=lambda t: -int(t[1]()["inst"]["L"][t[2]]) * t[3])
    fd = [t for t in tasks if t[0].startswith("tangent")]
    with ProcessPoolExecutor(max_workers=int(os.environ.get("GOLDEN_WORKERS", "7"))) as ex:
        # finite-difference jobs one at a time, their ten solves in parallel
        for t in fd:
            print(fd_one(t, ex), flush=True)
        for msg in ex.map(one, plain):
            print(msg, flush=True)
        for msg in ex.map(fv_one, fvt):
            print(msg, flush=True)
