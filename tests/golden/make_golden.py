"""Write oracle reference outputs for the parity tests (calls only oracle/ and workloads/).

Each file holds, for one instance of a named workload: m [N_s, 3], Phi [K_h+1, 3]
(complex), the Radau refinement r used and the change against the run with r/2
(time-discretisation error estimate).  Run:  python tests/golden/make_golden.py [names...]
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

def wide_l17():
    return W.small_random(2, 17, seed=117, samples=48, settle=1, n_harm=8)


def wide_l20():
    return W.small_random(2, 20, seed=120, samples=48, settle=1, n_harm=8)


def wide_l24():
    return W.small_random(2, 24, seed=124, samples=48, settle=1, n_harm=8)


# (workload factory, instance ids, Radau steps per sample for the reference and its check)
JOBS = {
    "wide_l17": (wide_l17, [0], 8),
    "wide_l20": (wide_l20, [0, 1], 8),
    "wide_l24": (wide_l24, [0, 1], 8),
    "single_1d": (W.single_1d, [0], 8),
    "lissajous": (W.lissajous_grid, [(0 * 17 + 8) * 17 + 8, (3 * 17 + 2) * 17 + 13, (5 * 17 + 16) * 17 + 0,
                                     (7 * 17 + 10) * 17 + 4, (2 * 17 + 0) * 17 + 16, (6 * 17 + 12) * 17 + 12], 4),
}


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
        factory, ids, r = JOBS[nm]
        tasks += [(nm, factory, i, r) for i in ids]
    with ProcessPoolExecutor(max_workers=min(7, len(tasks))) as ex:
        for msg in ex.map(one, tasks):
            print(msg, flush=True)
