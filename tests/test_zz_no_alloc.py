"""GPU test of fpn_solve_static, the solve that allocates nothing (its buffers live in a fixed device
array of the library): through the C ABI it gives the outputs of fpn_solve on the same inputs, bit for
bit (the same kernels run), and therefore within the 1e-5 parity bar of fpn_solve, on two calls in a
row, the second with fewer instances and fewer samples.  Requests beyond its limits, mixed degrees
and a context without the tables of the degree are rejected before any launch."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpn():
    import paper_2106_08040_amd as fpn
    return fpn


def _drive(fpn, ws):
    d = ws["drive"]
    return fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"])


def _np(x):
    return x.cpu().numpy() if x is not None else None


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_static_solve_matches_fpn_solve(fpn):
    import torch
    ctx = fpn.Context(0)
    try:
        for n, Ns, L in ((96, 48, 12), (37, 32, 12)):   # second call: smaller input
            ws = W.small_random(n, L, seed=600 + n, samples=Ns, settle=1, n_harm=6)
            args = (ws["inst"], ws["inst"]["L"], _drive(fpn, ws), Ns, 1, 6)
            m0, h0, s0 = ctx.solve(*args, harm_z=True)          # builds tables / twiddles
            m1, h1, s1 = ctx.solve_static(*args, harm_z=True)
            torch.cuda.synchronize()
            m0, h0, s0, m1, h1, s1 = (_np(x) for x in (m0, h0, s0, m1, h1, s1))
            print(f"n={n} Ns={Ns}: status {dict(zip(*np.unique(s1, return_counts=True)))}", flush=True)
            assert np.array_equal(s0, s1)
            assert np.array_equal(m0, m1, equal_nan=True) and np.array_equal(h0, h1, equal_nan=True)
            ok = np.isin(s0, [fpn.FPN_INST_OK, fpn.FPN_INST_TOL_UNMET])   # finished, outputs written
            assert ok.mean() > 0.8
            assert rel(m1[ok], m0[ok]) <= 1e-5 and rel(h1[ok], h0[ok]) <= 1e-5
        # only the samples: harmonics not requested, m given
        ws = W.small_random(5, 12, seed=605, samples=32, settle=1, n_harm=6)
        args = (ws["inst"], ws["inst"]["L"], _drive(fpn, ws), 32, 1, 6)
        m0, _, s0 = ctx.solve(*args, want_harm=False)
        m1, _, s1 = ctx.solve_static(*args, want_harm=False)
        torch.cuda.synchronize()
        assert np.array_equal(_np(m0), _np(m1), equal_nan=True) and np.array_equal(_np(s0), _np(s1))
    finally:
        ctx.close()


def test_static_solve_rejects_what_it_cannot_do(fpn):
    ctx = fpn.Context(0)
    try:
        ws = W.small_random(4, 10, seed=607, samples=32, settle=1, n_harm=4)
        args = (ws["inst"], ws["inst"]["L"], _drive(fpn, ws), 32, 1, 4)
        with pytest.raises(fpn.FpnError) as e:           # no tables of L = 10 in this context yet
            ctx.solve_static(*args)
        assert e.value.code == fpn.FPN_E_ARG
        ctx.solve(*args)
        big = W.small_random(fpn.FPN_STATIC_MAX_N + 1, 10, seed=608, samples=32, settle=1, n_harm=4)
        with pytest.raises(fpn.FpnError) as e:
            ctx.solve_static(big["inst"], big["inst"]["L"], _drive(fpn, big), 32, 1, 4)
        assert e.value.code == fpn.FPN_E_RANGE
        mixed = dict(ws)
        mixed["inst"] = {k: v.copy() for k, v in ws["inst"].items()}
        mixed["inst"]["L"][1] = 8
        with pytest.raises(fpn.FpnError) as e:
            ctx.solve_static(mixed["inst"], mixed["inst"]["L"], _drive(fpn, ws), 32, 1, 4)
        assert e.value.code == fpn.FPN_E_ARG
        with pytest.raises(fpn.FpnError) as e:
            ctx.solve_static(*args[:3], fpn.FPN_STATIC_MAX_NS + 2, 1, 4)
        assert e.value.code == fpn.FPN_E_RANGE
        w17 = W.small_random(2, 17, seed=609, samples=32, settle=1, n_harm=4)
        with pytest.raises(fpn.FpnError) as e:
            ctx.solve_static(w17["inst"], w17["inst"]["L"], _drive(fpn, w17), 32, 1, 4)
        assert e.value.code == fpn.FPN_E_RANGE
    finally:
        ctx.close()
