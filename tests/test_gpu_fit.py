"""GPU parity of the model fits and the distance measure (fpn_fit_rows, fpn_nrmse_global) against the
FP64 oracle (oracle/fit_oracle.py) on the same seeded synthetic system matrices, and the model-M1
pipeline end to end (solver -> closed-form scale -> NRMSE) against the oracle's pipeline on a small
dictionary.

Tolerance: both sides sum in FP64 over FP32 inputs; the GPU rounds its outputs to FP32, so a and the
NRMSE agree to a few FP32 ulps (asserted at 2e-6 relative)."""
import numpy as np
import pytest

import oracle as O
from oracle import fit_oracle as F
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


def oracle_rows(phi, S, pp, ps):
    """oracle a and Eq. error1 rows for every pair, from [.., n_pos, n_ch, n_bins] arrays."""
    A, E = [], []
    for i, j in zip(pp, ps):
        Fm = np.moveaxis(phi[i].astype(complex), 0, -1)   # [n_ch, n_bins, n_pos]
        Sm = np.moveaxis(S[j].astype(complex), 0, -1)
        a = F.fit_scaling(Fm, Sm)
        A.append(a)
        E.append(F.nrmse_rows(Sm, a[..., None] * Fm))
    return np.array(A), np.array(E)


def test_fit_rows_match_oracle(fpn, ctx):
    import torch
    phi = W.random_system_matrices(6, 121, 2, 37, seed=1)
    S = W.random_system_matrices(3, 121, 2, 37, seed=2)
    # an exactly scaled measurement, a zero dictionary row, tiny and huge rows
    S[2] = (phi[4].astype(complex) * (0.5 - 2j)).astype(np.complex64)
    phi[1][:, 0, 5] = 0
    phi[3][:, 1, :] *= 1e-6
    S[1][:, 0, :] *= 1e4
    pp = np.repeat(np.arange(6), 3)
    ps = np.tile(np.arange(3), 6)
    a, err = ctx.fit_rows(torch.tensor(phi, device="cuda:0"), torch.tensor(S, device="cuda:0"), pp, ps)
    a, err = a.cpu().numpy(), err.cpu().numpy()
    ar, er = oracle_rows(phi, S, pp, ps)
    scale = np.abs(ar) + 1e-30
    print(f"a max rel {np.max(np.abs(a - ar) / scale):.2e}, err max rel {np.max(np.abs(err - er) / er):.2e}", flush=True)
    assert np.all(np.abs(a - ar) <= 2e-6 * scale + 1e-30)
    assert np.all(np.abs(err - er) <= 2e-6 * er)
    # the zero row: a = 0 and eps = ||S|| / sqrt(N) / max|S|
    assert np.all(a[pp == 1][:, 0, 5] == 0)
    # the exactly scaled pair (phi 4, S 2): a = 0.5 - 2i up to FP32 rounding of S
    k = int(np.nonzero((pp == 4) & (ps == 2))[0][0])
    assert np.allclose(a[k], 0.5 - 2j, rtol=1e-6) and np.all(err[k] < 1e-6)


def test_nrmse_global_matches_oracle(fpn, ctx):
    import torch
    r = np.random.default_rng(3)
    n_groups, n_ang, n_ch, n_bins = 7, 12, 2, 101
    err = r.uniform(0.0, 0.5, (n_groups * n_ang, n_ch, n_bins)).astype(np.float32)
    kset = F.frequency_index_set(3, 3)
    ef, eg = ctx.nrmse_global(torch.tensor(err, device="cuda:0"), n_ang, kset)
    ef, eg = ef.cpu().numpy(), eg.cpu().numpy()
    for g in range(n_groups):
        e = err[g * n_ang:(g + 1) * n_ang].astype(float)
        efr = F.eps_freq(e[:, :, kset])
        assert np.allclose(ef[g], efr, rtol=2e-6, atol=0)
        assert abs(eg[g] - F.eps_global(efr)) <= 2e-6 * F.eps_global(efr)


def test_fit_argument_errors(fpn, ctx):
    import ctypes
    import torch
    x = torch.zeros((1, 4, 2, 3, 2), dtype=torch.float32, device="cuda:0")
    p = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    code = fpn._lib.fpn_fit_rows(ctx._h, x.data_ptr(), x.data_ptr(), 4, 2, 3, 1, p.data_ptr(), p.data_ptr(), None, None,
                                 None)
    assert code == fpn.FPN_E_ARG
    code = fpn._lib.fpn_fit_rows(ctx._h, x.data_ptr(), x.data_ptr(), 0, 2, 3, 1, p.data_ptr(), p.data_ptr(),
                                 x.data_ptr(), None, None)
    assert code == fpn.FPN_E_ARG
    code = fpn._lib.fpn_nrmse_global(ctx._h, x.data_ptr(), 1, 1, 2, 3, p.data_ptr(), 0, x.data_ptr(), None, None)
    assert code == fpn.FPN_E_ARG


def test_m1_pipeline_matches_oracle_pipeline(fpn, ctx):
    """A small M1 identification: a 2 x 2 dictionary (D, K) x 2 angles x 3 x 3 offsets on a short drive
    at L = 8; the "measurement" is the oracle's solve of an off-grid particle times a synthetic transfer
    value plus 1 % noise.  The GPU solves the dictionary and fits; the oracle solves the same dictionary
    and fits.  a, the row errors and the global NRMSE agree to the solver's 1e-5 level, and both pick
    the same (D, K)."""
    import torch
    base = W.small_random(1, 8, seed=7, samples=48, settle=1, n_harm=12)
    drive, Ns, Kh = base["drive"], 48, 12
    D_set, K_set, angles = (18e-9, 22e-9), (800.0, 2500.0), (20.0, 110.0)
    offs = [(x, y, 0.0) for y in (-5e-3, 0.0, 5e-3) for x in (-5e-3, 0.0, 5e-3)]
    rows = [(D, K, a) for D in D_set for K in K_set for a in angles]

    def instset(elems):
        n = len(elems) * len(offs)
        D = np.repeat([e[0] for e in elems], len(offs))
        K = np.repeat([e[1] for e in elems], len(offs))
        th = np.deg2rad(np.repeat([e[2] for e in elems], len(offs)))
        easy = np.stack([np.cos(th), np.sin(th), np.zeros(n)], 1)
        return dict(D=D, Ms=np.full(n, W.MAGNETITE_MS), K=K, alpha=np.full(n, 0.1), T=np.full(n, W.ROOM_T),
                    easy_axis=easy, offset=np.tile(np.array(offs), (len(elems), 1)), L=np.full(n, 8, np.int32))

    dic = instset(rows)
    truth = instset([(20.5e-9, 1300.0, a) for a in angles])

    def oracle_phi(inst):
        out = []
        for i in range(inst["D"].size):
            p = dict(D=inst["D"][i], Ms=inst["Ms"][i], K=inst["K"][i], alpha=inst["alpha"][i], T=inst["T"][i])
            o = O.solve_instance(p, inst["easy_axis"][i], 8, drive, Ns, 1, Kh, r=8, offset=inst["offset"][i])
            out.append(o["Phi"][:, :2].T)   # [ch, bins]
        return np.array(out)

    phi_o = oracle_phi(dic).reshape(len(rows), len(offs), 2, Kh + 1)
    S0 = oracle_phi(truth).reshape(len(angles), len(offs), 2, Kh + 1)
    a_true, z, rn = W.m1_transfer_and_noise(len(angles), len(offs), 2, Kh + 1, seed=70)
    S = a_true[None, None] * S0
    rms = np.sqrt(np.mean(np.abs(S) ** 2, axis=1, keepdims=True))
    S = (S + rn * rms * z).astype(np.complex64)
    pp = np.arange(len(rows))
    ps = np.tile(np.arange(len(angles)), len(rows) // len(angles))
    kset = np.arange(1, Kh + 1)
    # oracle pipeline (FP64 throughout)
    ar, er = oracle_rows(phi_o, S, pp, ps)
    egr = np.array([F.eps_global(F.eps_freq(er[g * 2:(g + 1) * 2][:, :, kset])) for g in range(len(rows) // 2)])
    # GPU pipeline
    d = fpn.make_drive(drive["amp"], drive["freq"], drive["period"], drive["phase"])
    _, h, st = ctx.solve(dic, dic["L"], d, Ns, 1, Kh, substeps=32, want_m=False)
    assert (st.cpu().numpy() == 0).all()
    phi_g = h.reshape(len(rows), len(offs), 2, Kh + 1)
    a, err = ctx.fit_rows(phi_g, torch.tensor(S, device="cuda:0"), pp, ps)
    ef, eg = ctx.nrmse_global(err, len(angles), kset)
    a, err, eg = a.cpu().numpy(), err.cpu().numpy(), eg.cpu().numpy()
    print("eps_global GPU", eg, "oracle", egr, flush=True)
    sel = np.abs(ar) > 1e-3 * np.abs(ar).max()
    assert np.max(np.abs(a - ar)[sel] / np.abs(ar)[sel]) < 1e-4
    assert np.max(np.abs(err - er)[:, :, kset] / er[:, :, kset]) < 1e-4
    assert np.allclose(eg, egr, rtol=1e-5)
    assert int(np.argmin(eg)) == int(np.argmin(egr))


def test_m2_system_model_and_rows_error_match_oracle(fpn, ctx):
    """fpn_m2_system (G = M^H M, b = M^H y, ||y||^2 of the weighted M2 dictionary), fpn_m2_model and
    fpn_rows_error against the oracle's M2 system, model and Eq. error1 on seeded synthetic inputs."""
    import torch
    J, n_ang, n_pos, n_ch, n_bins = 5, 3, 25, 2, 20
    phi = W.random_system_matrices(J * n_ang, n_pos, n_ch, n_bins, seed=11)
    a = W.random_system_matrices(1, J * n_ang, n_ch, n_bins, seed=12)[0]
    S = W.random_system_matrices(n_ang, n_pos, n_ch, n_bins, seed=13)
    kset = np.array([1, 4, 5, 9, 17])
    dev = "cuda:0"
    G, b, yy = ctx.m2_system(torch.tensor(phi, device=dev), torch.tensor(a, device=dev), torch.tensor(S, device=dev),
                             n_ang, kset)
    G, b, yy = G.cpu().numpy(), b.cpu().numpy(), float(yy.cpu().numpy()[0])
    # oracle: Psi [J, angles, channels, bins, N] = a * Phi
    ph = phi.astype(complex).reshape(J, n_ang, n_pos, n_ch, n_bins).transpose(0, 1, 3, 4, 2)
    av = a.astype(complex).reshape(J, n_ang, n_ch, n_bins)
    Psi = av[..., None] * ph
    Sm = S.astype(complex).transpose(0, 2, 3, 1)
    M, y = F.m2_system(Psi, Sm, kset)
    Gr, br, yyr = M.conj().T @ M, M.conj().T @ y, float(np.vdot(y, y).real)
    print(f"G {np.abs(G - Gr).max() / np.abs(Gr).max():.2e}  b {np.abs(b - br).max() / np.abs(br).max():.2e}  "
          f"yy {abs(yy - yyr) / yyr:.2e}", flush=True)
    assert np.abs(G - Gr).max() <= 1e-6 * np.abs(Gr).max()
    assert np.abs(b - br).max() <= 1e-6 * np.abs(br).max()
    assert abs(yy - yyr) <= 1e-6 * yyr
    w = np.array([0.5, 0.0, 1.25, 2.0, 0.1])
    model = ctx.m2_model(torch.tensor(phi, device=dev), torch.tensor(a, device=dev), w, n_ang)
    mref = F.m2_model(Psi, w)                       # [angles, channels, bins, N]
    mg = model.cpu().numpy().astype(complex).transpose(0, 2, 3, 1)
    assert np.abs(mg - mref).max() <= 2e-6 * np.abs(mref).max()
    err = ctx.rows_error(model, torch.tensor(S, device=dev)).cpu().numpy()
    eref = F.nrmse_rows(Sm, mref)
    assert np.allclose(err, eref, rtol=2e-6)


def test_m2_weights_from_device_system_match_oracle(fpn, ctx):
    """The M2 weights from the device-formed system (fpn_m2_system, then fpn_m2_weights on the host)
    against the oracle's SVD + NNLS on the same seeded dictionary: truncated objective and, untruncated,
    the weights."""
    import torch
    J, n_ang, n_pos, n_ch, n_bins = 6, 2, 30, 2, 12
    phi = W.random_system_matrices(J * n_ang, n_pos, n_ch, n_bins, seed=21)
    a = W.random_system_matrices(1, J * n_ang, n_ch, n_bins, seed=22)[0]
    # a measurement that is a noisy non-negative superposition of the dictionary
    ph = phi.astype(complex).reshape(J, n_ang, n_pos, n_ch, n_bins)
    av = a.astype(complex).reshape(J, n_ang, 1, n_ch, n_bins)
    wt = np.array([0.7, 0.0, 1.1, 0.0, 0.4, 0.9])
    S = (np.tensordot(wt, av * ph, axes=(0, 0)) + 0.2 * W.random_system_matrices(n_ang, n_pos, n_ch, n_bins, seed=23)
         ).astype(np.complex64)
    kset = np.arange(1, n_bins)
    dev = "cuda:0"
    G, b, yy = ctx.m2_system(torch.tensor(phi, device=dev), torch.tensor(a, device=dev), torch.tensor(S, device=dev),
                             n_ang, kset)
    G, b, yy = G.cpu().numpy(), b.cpu().numpy(), float(yy.cpu().numpy()[0])
    Psi = av.transpose(0, 1, 3, 4, 2) * ph.transpose(0, 1, 3, 4, 2)
    M, y = F.m2_system(Psi, S.astype(complex).transpose(0, 2, 3, 1), kset)
    for s in (0, 4):
        w, full, red, rank = fpn.m2_weights(G, b, yy, s=s)
        wo, fullo, redo = F.m2_weights(M, y, s=None if s == 0 else s)
        print(f"s={s}: rank {rank}, objective {red:.6e} vs oracle {redo:.6e}", flush=True)
        assert abs(red - redo) <= 1e-5 * yy
        if s == 0:
            assert np.allclose(w, wo, atol=1e-4 * wo.max())
