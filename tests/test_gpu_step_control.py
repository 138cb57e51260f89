"""GPU regression tests of the per-step error control.

* Particles at the edge of resolution (the L = 24 particles of the uneven sweep, sigma up to 20):
  every sample interval must finish in a bounded number of RODAS4 steps.  A rejected step that the
  landing rule stretched back to the same length was once retried until the error estimate happened
  to fall below the tolerance.
* Large particles in strong transverse fields (the identification problem's components at positive
  y offsets): an attempted step one sample spacing long overflows the FP32 factorisation.  Such an
  attempt was once taken as a failure of the instance; it is rejected and retried shorter, and the
  results match the FP64 oracle.
"""
import glob
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_overflowing_attempts_are_retried():
    """Every instance finishes and the oracle's three instances are within 1e-5.  The third (component 2,
    sigma = 11, in the strongest field of the grid: offset (12, 12) mT) was at 3.3e-5 on Phi while the
    Schur blocks were inverted without pivoting (growth factor ~5e3 at a step one sample spacing long);
    with partial pivoting it meets the same bound as the others."""
    import torch

    import paper_2106_08040_amd as fpn
    ws = W.identification_problem()
    full = W.identification_instances(ws, 0)
    files = sorted(glob.glob(os.path.join(GOLDEN, "identification_a0_*.npz")))
    gold = [int(np.load(f)["idx"]) for f in files]
    # every 8th offset with y > 0 (offset index >= 512), all four components, plus the oracle's instances
    idx = [o * 4 + c for o in range(512, 1024, 8) for c in range(4)] + gold
    sub = W.take(full, idx)
    d = sub["drive"]
    ctx = fpn.Context(0)
    try:
        drive = fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"])
        m, h, st = ctx.solve(sub["inst"], sub["inst"]["L"], drive, sub["samples"], sub["settle"], 64)
        torch.cuda.synchronize()
        m, h, st = m.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    finally:
        ctx.close()
    print(f"{len(idx)} instances: status {dict(zip(*np.unique(st, return_counts=True)))}, "
          f"max |m| {np.linalg.norm(m, axis=1).max():.4f}", flush=True)
    assert (st == 0).all() and np.isfinite(m).all() and np.isfinite(h).all()
    assert np.linalg.norm(m, axis=1).max() <= 1.0 + 1e-3
    if not files:
        pytest.skip("no golden files (run tests/golden/make_golden.py identification_a0)")
    for k, f in enumerate(files):
        g = np.load(f)
        j = len(idx) - len(gold) + k
        # change of the reference against the run with half the Radau IIA steps: its own error is this
        # change / (2^3 - 1) or less (stiff order 3), far below the bounds below
        assert g["err_est"] < 3e-6
        em, eh = rel(m[j].T, g["m"]), rel(h[j].T, g["Phi"][:, :2])
        print(f"identification inst {gold[k]}: m {em:.2e} Phi {eh:.2e}", flush=True)
        assert em < 1e-5 and eh < 1e-5


def test_hard_particles_finish_in_bounded_steps():
    """The L = 24 particles of the uneven sweep (sigma up to 67: above 20 no degree up to 24 resolves
    them) on a short three-axis drive: every instance ends OK, TOL_UNMET or UNRESOLVED; those that run
    to the end take a bounded number of steps per sample interval and have |m| <= 1 + 1e-3; the
    unresolvable ones are flagged, not returned as OK."""
    import torch

    import paper_2106_08040_amd as fpn
    ws = W.uneven_sweep(4096, seed=3)
    sub = W.take(ws, np.nonzero(ws["inst"]["L"] == 24)[0])
    ok_rule = W.resolvable(sub["inst"]["D"], sub["inst"]["K"], sub["inst"]["L"])
    ctx = fpn.Context(0)
    try:
        T = 40e-6
        drive = fpn.make_drive((10e-3, 8e-3, 0.0), (3 / T, 4 / T, 0.0), T, (0.0, 0.3, 0.0))
        Ns = 64
        p = ctx.plan(sub["inst"], sub["inst"]["L"], drive, Ns, 1, 8, want_m=True)
        p.launch()
        torch.cuda.synchronize()
        per_interval = p.steps() / (2 * Ns)
        status = p.status.cpu().numpy()
        m = p.m.cpu().numpy()
        p.close()
    finally:
        ctx.close()
    done = (status == fpn.FPN_INST_OK) | (status == fpn.FPN_INST_TOL_UNMET)
    print(f"{len(status)} particles ({ok_rule.sum()} resolvable by the degree rule): status "
          f"{dict(zip(*np.unique(status, return_counts=True)))}; finished: steps per sample interval mean "
          f"{per_interval[done].mean():.1f}, max {per_interval[done].max():.1f}", flush=True)
    assert np.isin(status, [fpn.FPN_INST_OK, fpn.FPN_INST_TOL_UNMET, fpn.FPN_INST_UNRESOLVED]).all()
    assert np.isfinite(m[done]).all() and np.isnan(m[~done]).all()
    assert np.linalg.norm(m[done], axis=1).max() <= 1.0 + 1e-3
    # the smallest step is 1/64 of the sample spacing; rejections may add to that, not multiply it
    assert per_interval[done].max() <= 128 and per_interval[done].mean() <= 64
