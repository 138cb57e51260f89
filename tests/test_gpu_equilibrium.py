"""GPU tests of the equilibrium model (model M0, Eq. Langevin) against the oracle: the 2312-instance
Lissajous system matrix in one call, every fourth instance checked, rel-L2 <= 1e-5 per instance on m and on Phi (FP64
evaluation on both sides, the GPU stores FP32), bad instances isolated, outputs independent of
whether m is requested."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_equilibrium_lissajous_matches_oracle():
    import torch

    import paper_2106_08040_amd as fpn
    ws = W.lissajous_grid()
    d = ws["drive"]
    ctx = fpn.Context(0)
    try:
        drive = fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"])
        m, h, st = ctx.equilibrium(ws["inst"], drive, ws["samples"], ws["settle"], ws["n_harm"])
        _, h2, _ = ctx.equilibrium(ws["inst"], drive, ws["samples"], ws["settle"], ws["n_harm"], want_m=False)
        torch.cuda.synchronize()
        m, h, st, h2 = m.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy(), h2.cpu().numpy()
    finally:
        ctx.close()
    assert (st == 0).all() and np.array_equal(h, h2)
    inst = ws["inst"]
    worst = [0.0, 0.0]
    sample = list(range(0, inst["D"].size, 4)) + [inst["D"].size - 1]  # the whole batch runs; a quarter is checked
    for i in sample:
        p = dict(D=inst["D"][i], Ms=inst["Ms"][i], K=inst["K"][i], alpha=inst["alpha"][i], T=inst["T"][i])
        ref = O.equilibrium_instance(p, d, ws["samples"], ws["settle"], ws["n_harm"], offset=inst["offset"][i])
        em, eh = rel(m[i].T, ref["m"]), rel(h[i].T, ref["Phi"][:, :2])
        worst = [max(worst[0], em), max(worst[1], eh)]
        assert em < TOL and eh < TOL, (i, em, eh)
    print(f"{len(sample)} of 2312 instances: worst rel-L2 m {worst[0]:.2e} Phi {worst[1]:.2e}", flush=True)


def test_equilibrium_bad_instance_is_isolated():
    import torch

    import paper_2106_08040_amd as fpn
    ws = W.small_random(4, 10, seed=9)
    ws["inst"]["D"] = ws["inst"]["D"].copy()
    ws["inst"]["D"][1] = -1.0
    d = ws["drive"]
    ctx = fpn.Context(0)
    try:
        drive = fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"])
        m, h, st = ctx.equilibrium(ws["inst"], drive, ws["samples"], ws["settle"], ws["n_harm"], harm_z=True)
        torch.cuda.synchronize()
        m, h, st = m.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()
    finally:
        ctx.close()
    assert st[1] == fpn.FPN_INST_BAD_PARAM and np.isnan(m[1]).all() and np.isnan(h[1]).all()
    assert (st[[0, 2, 3]] == 0).all()
    for i in (0, 2, 3):
        inst = {k: v[i] for k, v in ws["inst"].items()}
        p = dict(D=inst["D"], Ms=inst["Ms"], K=inst["K"], alpha=inst["alpha"], T=inst["T"])
        ref = O.equilibrium_instance(p, d, ws["samples"], ws["settle"], ws["n_harm"], offset=inst["offset"])
        assert rel(m[i].T, ref["m"]) < TOL and rel(h[i].T, ref["Phi"]) < TOL
