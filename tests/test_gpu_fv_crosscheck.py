"""The GPU Galerkin path against an independent discretisation (finite volumes, oracle/fv_oracle.py).

Parity tests compare the GPU with the Galerkin oracle at the same degree L, so both carry the same
truncation error.  Here the reference is the finite-volume solution of Eq. FP-general on the refined
icosahedron, extrapolated from 5120 and 20480 triangles (second order in the mesh width), stored by
tests/golden/make_golden.py ("fv"): the GPU solution at a degree high enough for these particles
must reach it to within the reference's own error (its extrapolation change and its BDF2 time
error), and the GPU solution at the degree of the sweeps' degree rule must match the Galerkin oracle
at that degree (parity) while its distance to the reference measures the truncation error of the
rule, which the test reports and bounds from below and above.
"""
import glob
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def reference(z):
    """Extrapolated finite-volume moment and a bound on its error (extrapolation change + time error)."""
    R45 = (4 * z["fv5"] - z["fv4"]) / 3
    R34 = (4 * z["fv4"] - z["fv3"]) / 3
    e_space = rel(R45, R34)
    e_time = rel(z["fv4"], z["fv4_half_r"]) / 3     # BDF2: error at r ~ (change from r/2) / 3
    return R45, e_space + e_time


@pytest.fixture(scope="module")
def solved():
    import torch
    import paper_2106_08040_amd as fpn
    files = sorted(glob.glob(os.path.join(GOLDEN, "fv_*.npz")))
    if not files:
        pytest.skip("no finite-volume golden files (run tests/golden/make_golden.py fv)")
    ws = W.fv_crosscheck()
    d = ws["drive"]
    ctx = fpn.Context(0)
    drive = fpn.make_drive(d["amp"], d["freq"], d["period"], d["phase"])
    out = {}
    for tag, dL in (("rule", 0), ("high", 6)):
        L = ws["inst"]["L"] + dL
        m, h, st = ctx.solve(ws["inst"], L, drive, ws["samples"], ws["settle"], ws["n_harm"], harm_z=True)
        torch.cuda.synchronize()
        out[tag] = (m.cpu().numpy(), st.cpu().numpy())
    ctx.close()
    return files, out


def test_gpu_converges_to_the_finite_volume_solution(solved):
    files, out = solved
    m, st = out["high"]
    for f in files:
        z = np.load(f)
        i = int(z["idx"])
        R, err = reference(z)
        got = m[i].T                                   # [3][N_s] -> [N_s][3]
        e = rel(got, R)
        print(f"instance {i}: L + 6 = {int(z['L']) + 6}, GPU vs finite volumes {e:.2e}, reference error {err:.1e}")
        assert st[i] == 0
        assert e <= 2.0 * err + 1e-5


def test_degree_rule_truncation_is_measured(solved):
    """At the rule's degree the GPU matches the Galerkin oracle at that degree (parity, 1e-5), and its
    distance to the finite-volume reference equals the oracle's truncation error (the change from L
    to L + 6) to within the reference's error."""
    files, out = solved
    m, st = out["rule"]
    for f in files:
        z = np.load(f)
        i = int(z["idx"])
        R, err = reference(z)
        got = m[i].T
        assert st[i] == 0
        assert rel(got, z["gal_L"]) <= 1e-5
        trunc = rel(z["gal_L"], z["gal_L6"])
        e = rel(got, R)
        print(f"instance {i}: L = {int(z['L'])}, truncation {trunc:.2e}, GPU vs finite volumes {e:.2e}")
        assert abs(e - trunc) <= 2.0 * err + 2e-5
