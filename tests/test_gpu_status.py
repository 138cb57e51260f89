"""GPU tests of per-instance statuses and of context-owned tables that plans keep.

* A particle far beyond what its Galerkin degree resolves (sigma = 69 at L = 8: the truncated
  operator has growing modes) ends FPN_INST_UNRESOLVED or FPN_INST_NONFINITE with NaN outputs, and
  does not disturb a resolved instance of the same batch, which matches its own single-instance solve.
* Twiddle tables are kept per sample count: a plan built for N_s = 32 still gives the eager N_s = 32
  result, launched directly and through its graph, after solves with N_s = 48 and 96 in between.
* Sample counts beyond the harmonics reduction's LDS limit are rejected with FPN_E_RANGE.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpn():
    import paper_2106_08040_amd as fpn
    return fpn


@pytest.fixture(scope="module")
def ctx(fpn):
    c = fpn.Context(0)
    yield c
    c.close()


def solve(fpn, ctx, ws, samples=None, n_harm=None, substeps=0):
    import torch
    d = ws["drive"]
    drive = fpn.make_drive(d["amp"], d["freq"], d["period"], d.get("phase", (0, 0, 0)))
    m, h, st = ctx.solve(ws["inst"], ws["inst"]["L"], drive, samples or ws["samples"], ws["settle"],
                         n_harm if n_harm is not None else ws["n_harm"], substeps=substeps, harm_z=ws["harm_z"])
    torch.cuda.synchronize()
    return m.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()


def test_unresolvable_particle_is_flagged(fpn, ctx):
    ws = W.small_random(2, 8, seed=71, samples=32, settle=1, n_harm=6)
    ws["inst"] = {k: v.copy() for k, v in ws["inst"].items()}
    inst = ws["inst"]
    inst["D"][0], inst["K"][0] = 30e-9, 2e4    # sigma = 69.4
    assert W.anisotropy_ratio(inst["D"][0], inst["K"][0]) > 60 and W.resolvable(inst["D"][1], inst["K"][1], 8)
    m, h, st = solve(fpn, ctx, ws)
    print(f"status {st.tolist()}", flush=True)
    assert st[0] in (fpn.FPN_INST_UNRESOLVED, fpn.FPN_INST_NONFINITE)
    assert np.isnan(m[0]).all() and np.isnan(h[0]).all()
    assert st[1] in (fpn.FPN_INST_OK, fpn.FPN_INST_TOL_UNMET)
    m1, h1, st1 = solve(fpn, ctx, W.take(ws, [1]))
    assert np.array_equal(m1[0], m[1]) and np.array_equal(h1[0], h[1])


def test_plan_keeps_its_twiddle_table(fpn, ctx):
    import torch
    ws = W.small_random(3, 10, seed=72, samples=32, settle=1, n_harm=6)
    d = ws["drive"]
    drive = fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"])
    p = ctx.plan(ws["inst"], ws["inst"]["L"], drive, 32, 1, 6, substeps=2, want_m=True, harm_z=True)
    try:
        m_ref, h_ref, st = solve(fpn, ctx, ws, 32, 6, substeps=2)
        assert (st == 0).all()
        for Ns in (48, 96):                                  # other tables made after the plan's
            solve(fpn, ctx, ws, Ns, 6, substeps=2)
        for launch in (p.launch, p.graph_launch, p.launch, p.graph_launch):
            p.m.zero_()
            launch()
            torch.cuda.synchronize()
            assert np.array_equal(p.m.cpu().numpy(), m_ref)
            assert np.array_equal(p.harm.cpu().numpy(), h_ref)
            solve(fpn, ctx, ws, 48, 6, substeps=2)            # eager work between the launches
    finally:
        p.close()


def test_sample_count_beyond_harmonics_lds_is_rejected(fpn, ctx):
    ws = W.small_random(1, 6, seed=73, samples=32, settle=0, n_harm=4)
    d = ws["drive"]
    drive = fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"])
    with pytest.raises(fpn.FpnError) as e:
        ctx.solve(ws["inst"], ws["inst"]["L"], drive, 8193, 0, 4, substeps=1, harm_z=False)
    assert e.value.code == fpn.FPN_E_RANGE
    with pytest.raises(fpn.FpnError) as e:
        ctx.solve(ws["inst"], ws["inst"]["L"], drive, 5462, 0, 4, substeps=1, harm_z=True)
    assert e.value.code == fpn.FPN_E_RANGE
