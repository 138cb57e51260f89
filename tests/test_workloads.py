"""CPU tests of the seeded input generators: sizes, index maps, ranges and determinism."""
import numpy as np
import pytest

import workloads as W


def test_lissajous_grid_layout():
    ws = W.lissajous_grid()
    inst = ws["inst"]
    assert inst["D"].size == 2312 and (inst["L"] == 16).all()
    offs = np.linspace(-12e-3, 12e-3, 17)
    for j, iy, ix in ((0, 0, 0), (3, 5, 16), (7, 16, 16)):
        i = (j * 17 + iy) * 17 + ix
        assert np.allclose(inst["offset"][i], [offs[ix], offs[iy], 0.0], rtol=0, atol=1e-15)
        assert np.allclose(inst["easy_axis"][i], [np.cos(j * np.pi / 8), np.sin(j * np.pi / 8), 0.0])
    # 16 and 17 drive cycles per repetition time (the mixing orders of the Lissajous trajectory)
    assert ws["drive"]["period"] * np.array(ws["drive"]["freq"][:2]) == pytest.approx([16, 17], rel=1e-12)


def test_uneven_sweep_keeps_every_draw_and_is_seeded():
    """The sweep keeps the full D ~ U[15, 30] nm x K log-U[0.5, 20] kJ/m^3 distribution: the pairs that
    no degree up to 24 resolves (sigma > 20) stay in it at L = 24 and are told apart by `resolvable`."""
    a, b = W.uneven_sweep(4096, seed=3), W.uneven_sweep(4096, seed=3)
    for k in a["inst"]:
        assert np.array_equal(a["inst"][k], b["inst"][k])
    inst = a["inst"]
    sigma = W.anisotropy_ratio(inst["D"], inst["K"])
    assert inst["D"].min() >= 15e-9 and inst["D"].max() <= 30e-9
    assert inst["K"].min() >= 500 and inst["K"].max() <= 2e4
    assert sigma.max() > 60                       # the largest particles are kept
    assert inst["L"].min() == 8 and inst["L"].max() == 24
    assert (inst["L"] == np.clip(np.ceil(sigma) + 4, 8, 24)).all()
    ok = W.resolvable(inst["D"], inst["K"], inst["L"])
    assert np.array_equal(ok, sigma <= 20) and 0.8 < ok.mean() < 0.95
    assert np.allclose(np.linalg.norm(inst["easy_axis"], axis=1), 1.0)


def test_identification_problem_layout():
    ws = W.identification_problem()
    off, ang = ws["offsets"], ws["angles"]
    assert off.shape == (1024, 3) and ang.size == 16
    assert off[:, 0].min() == -12e-3 and np.isclose(off[:, 0].max(), 12e-3)
    assert np.allclose(off[33], [off[1, 0], off[32, 1], 0.0])      # offset index = iy * 32 + ix
    assert np.allclose(ang, np.arange(16) * np.pi / 16)
    t, g = ws["truth"], ws["guess"]
    assert ((t["D"] >= 16e-9) & (t["D"] <= 28e-9)).all() and ((t["K"] >= 500) & (t["K"] <= 5e3)).all()
    assert ((t["alpha"] >= 0.05) & (t["alpha"] <= 0.3)).all() and ((t["w"] >= 0.1) & (t["w"] <= 1)).all()
    # L = 16 meets the degree rule for the truth and for the point where the gradient is taken
    for p in (t, g):
        assert (np.ceil(W.anisotropy_ratio(p["D"], p["K"])) + 4 <= ws["L"]).all()
    n1, n2 = ws["noise_rng"]().normal(size=5), W.identification_problem()["noise_rng"]().normal(size=5)
    assert np.array_equal(n1, n2)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus N > 1 exits with status 2 and says why, before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_surrogate_particle_family_draws_and_grid():
    """Particle-family surrogate inputs: every draw is resolved by its degree (8..16), the (D, K, alpha)
    ranges are the uneven sweep's, axes are unit vectors (uniform on the sphere: mean near 0), and the
    evaluation grid is 8 sets x 64 Fibonacci axes x 64^2 offsets in the documented instance order."""
    inst = W.surrogate_particles(4096, 21)["inst"]
    assert inst["D"].size == 4096 and W.resolvable(inst["D"], inst["K"], inst["L"]).all()
    assert inst["L"].min() >= 8 and inst["L"].max() == 16
    assert ((inst["D"] >= 15e-9) & (inst["D"] <= 30e-9)).all() and ((inst["K"] >= 500) & (inst["K"] <= 2e4)).all()
    assert ((inst["alpha"] >= 0.05) & (inst["alpha"] <= 0.3)).all()
    assert np.allclose(np.linalg.norm(inst["easy_axis"], axis=1), 1.0)
    assert np.abs(inst["easy_axis"].mean(0)).max() < 0.05
    ax = W.fibonacci_axes(64)
    assert np.allclose(np.linalg.norm(ax, axis=1), 1.0) and np.abs(ax.mean(0)).max() < 0.02
    g = W.surrogate_particle_grid()["inst"]
    assert g["D"].size == 8 * 64 * 64 * 64
    assert np.unique(g["D"]).size == 8 and W.resolvable(g["D"], g["K"], g["L"]).all()
    i = 3 * 64 * 4096 + 5 * 4096 + 7 * 64 + 9          # set 3, axis 5, offset y 7, offset x 9
    step = 24e-3 / 64
    assert np.allclose(g["easy_axis"][i], ax[5])
    assert np.allclose(g["offset"][i], [-12e-3 + 9.5 * step, -12e-3 + 7.5 * step, 0.0])
    assert g["D"][i] == g["D"][3 * 262144] and g["D"][i] != g["D"][4 * 262144]
