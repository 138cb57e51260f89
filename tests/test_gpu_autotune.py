"""GPU tests of the launch-configuration autotuner (batching): every compiled workgroup size of the
register-layout stepper integrates each instance with one wavefront in the same order, so outputs do
not depend on the size; the autotuner picks a compiled size and the context then uses it."""
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


def _solve(fpn, ctx, ws):
    import torch
    d = ws["drive"]
    m, h, st = ctx.solve(ws["inst"], ws["inst"]["L"], fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"]),
                         ws["samples"], ws["settle"], ws["n_harm"], harm_z=True)
    torch.cuda.synchronize()
    return m.cpu().numpy(), h.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("L", [8, 12])
def test_every_workgroup_size_gives_the_same_outputs(fpn, ctx, L):
    ws = W.small_random(40, L, seed=900 + L, samples=48, settle=1, n_harm=6)
    ref = None
    for w in fpn.fpn_stepper_wave_options(L):
        ctx.set_stepper_waves(L, w)
        m, h, st = _solve(fpn, ctx, ws)
        assert np.isin(st, [fpn.FPN_INST_OK, fpn.FPN_INST_TOL_UNMET]).all()   # finished, outputs written
        if ref is None:
            ref = (m, h, st)
            continue
        assert np.array_equal(st, ref[2])
        dm = np.abs(m - ref[0]).max() / np.abs(ref[0]).max()
        dh = np.abs(h - ref[1]).max() / np.abs(ref[1]).max()
        print(f"L={L} waves={w}: max |dm| {dm:.1e}, max |dPhi| {dh:.1e} (relative to the largest entry)", flush=True)
        assert dm <= 1e-6 and dh <= 1e-6
    ctx.set_stepper_waves(L, 0)


def test_autotune_picks_a_compiled_size(fpn, ctx):
    L = 10
    w, ns = ctx.autotune(L)
    opts = fpn.fpn_stepper_wave_options(L)
    print("autotune L=10:", w, ns, flush=True)
    assert w in opts and set(ns) == set(opts)
    assert np.isfinite(ns[w]) and ns[w] > 0 and ns[w] == min(ns.values())
    ws = W.small_random(16, L, seed=77, samples=32, settle=1, n_harm=4)
    m, h, st = _solve(fpn, ctx, ws)  # the tuned size is the one in use
    ctx.set_stepper_waves(L, 0)
    m0, h0, st0 = _solve(fpn, ctx, ws)
    assert np.isin(st, [fpn.FPN_INST_OK, fpn.FPN_INST_TOL_UNMET]).all() and np.array_equal(st, st0)
    assert np.abs(m - m0).max() <= 1e-6 * np.abs(m0).max()


def test_wide_degree_autotune_has_one_configuration(fpn, ctx):
    w, ns = ctx.autotune(17)
    assert w == 0 and list(ns) == [0] and np.isfinite(ns[0])


def test_unknown_workgroup_size_is_rejected(fpn, ctx):
    with pytest.raises(fpn.FpnError):
        ctx.set_stepper_waves(16, 12)   # 12 is compiled for L <= 13 only
    with pytest.raises(fpn.FpnError):
        ctx.set_stepper_waves(8, 5)


@pytest.mark.parametrize("L", [17, 24])
def test_wide_layouts_give_the_same_outputs(fpn, ctx, L):
    """The wide layout (L = 17..24) keeps each instance's block inverses and stage vectors either in a
    global workspace (4 instances per workgroup) or in LDS (1 per workgroup); a plan picks one by its
    cost estimate, fpn_set_stepper_waves(L, 4 or 1) forces it.  Same arithmetic in the same order:
    the outputs are bitwise the same, and 0 hands the choice back to the plans."""
    ws = W.small_random(24, L, seed=950 + L, samples=32, settle=1, n_harm=6)
    out = {}
    try:
        for w in (4, 1, 0):
            ctx.set_stepper_waves(L, w)
            out[w] = _solve(fpn, ctx, ws)
    finally:
        ctx.set_stepper_waves(L, 0)
    assert np.isin(out[4][2], [fpn.FPN_INST_OK, fpn.FPN_INST_TOL_UNMET, fpn.FPN_INST_UNRESOLVED]).all()
    for w in (1, 0):
        for a, b in zip(out[4], out[w]):
            assert np.array_equal(a, b, equal_nan=True), w
    with pytest.raises(fpn.FpnError):
        ctx.set_stepper_waves(L, 8)
