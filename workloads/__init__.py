"""Seeded synthetic workloads (instance sets) shared by the tests, the bench and the oracle checks.

This module only draws and lays out inputs; it contains none of the solver's
arithmetic.  Shapes follow the paper's experiment (Experimental Setup and
Simulation Setting): a 2D Lissajous drive with f_x = 2.5 MHz / 102 and
f_y = 2.5 MHz / 96 (repetition time 652.8 us, 1632 samples at 2.5 MHz), easy axes
in the xy-plane at angles measured from x, offset (selection) fields on a regular
grid, particle diameters and anisotropies in the ranges of the simulation sets.
They stand in for the measured calibration data, which is not available.

Every instance set is a dict with SoA arrays (SI units, fields as mu0*H in tesla):
  D, Ms, K, alpha, T  [n]      easy_axis [n,3]   offset [n,3]   L [n] (int32)
plus the drive (amp, freq, phase, period) and the sampling options.
"""
import numpy as np

MAGNETITE_MS = 474e3      # A/m
ROOM_T = 295.0            # K
LISSAJOUS_T = 652.8e-6    # s
LISSAJOUS_F = (2.5e6 / 102, 2.5e6 / 96, 0.0)


def _instances(D, Ms, K, alpha, T, easy, offset, L):
    n = len(D)
    return dict(D=np.asarray(D, float), Ms=np.asarray(Ms, float), K=np.asarray(K, float),
                alpha=np.asarray(alpha, float), T=np.asarray(T, float),
                easy_axis=np.asarray(easy, float).reshape(n, 3), offset=np.asarray(offset, float).reshape(n, 3),
                L=np.asarray(L, np.int32).reshape(n))


def lissajous_drive(amp=(12e-3, 12e-3, 0.0)):
    return dict(amp=tuple(amp), freq=LISSAJOUS_F, phase=(0.0, 0.0, 0.0), period=LISSAJOUS_T)


def single_1d():
    """One instance: 1D drive along x, 12 mT at 25 kHz, zero offset, easy axis at 30 deg to x in the
    xy-plane, magnetite D = 20 nm, K = 2 kJ/m^3, alpha = 0.1, T = 295 K, L = 10, 3 periods with the
    last recorded at 1000 samples, harmonics 0..20 of x, y, z."""
    th = np.deg2rad(30.0)
    inst = _instances([20e-9], [MAGNETITE_MS], [2e3], [0.1], [ROOM_T], [[np.cos(th), np.sin(th), 0.0]],
                      [[0.0, 0.0, 0.0]], [10])
    drive = dict(amp=(12e-3, 0.0, 0.0), freq=(25e3, 0.0, 0.0), phase=(0.0, 0.0, 0.0), period=40e-6)
    return dict(name="single_1d_L10", inst=inst, drive=drive, samples=1000, settle=2, n_harm=20, harm_z=True)


def lissajous_grid(n_off=17, n_ang=8, L=16, span=12e-3):
    """2D Lissajous system matrix: 17 x 17 offsets on +-12 mT x 8 easy-axis angles j*pi/8 in the
    xy-plane; D = 20 nm, K = 2 kJ/m^3, alpha = 0.1, L = 16.  Instance id = (j*17 + iy)*17 + ix."""
    offs = -span + (2 * span / (n_off - 1)) * np.arange(n_off)
    j, iy, ix = np.meshgrid(np.arange(n_ang), np.arange(n_off), np.arange(n_off), indexing="ij")
    j, iy, ix = j.ravel(), iy.ravel(), ix.ravel()
    th = j * np.pi / n_ang
    n = th.size
    easy = np.stack([np.cos(th), np.sin(th), np.zeros(n)], 1)
    off = np.stack([offs[ix], offs[iy], np.zeros(n)], 1)
    inst = _instances(np.full(n, 20e-9), np.full(n, MAGNETITE_MS), np.full(n, 2e3), np.full(n, 0.1),
                      np.full(n, ROOM_T), easy, off, np.full(n, L))
    return dict(name=f"lissajous_{n_off}x{n_off}x{n_ang}_L{L}", inst=inst, drive=lissajous_drive(),
                samples=1632, settle=1, n_harm=200, harm_z=False)


def truncation_degree(D, K, T=ROOM_T, lo=8, hi=24):
    """Galerkin degree rule of the uneven sweep: L = clamp(ceil(sigma) + 4, lo, hi),
    sigma = K (pi D^3 / 6) / (k_B T); evaluated once here so every consumer reads the same integer.

    The truncated Galerkin operator acquires an eigenvalue with positive real part (a spurious
    growing mode) once sigma exceeds about L - 1 (scanned for L = 12..24, fields up to 24 mT,
    alpha 0.05..0.25), so the degree has to grow linearly with sigma; the margin of 4 keeps the
    operator stable up to sigma = 20 at L = 24.  Particles with larger sigma get L = hi and are not
    resolved by it (``resolvable`` is False for them)."""
    sigma = anisotropy_ratio(D, K, T)
    return np.clip(np.ceil(sigma) + 4, lo, hi).astype(np.int32)


def resolvable(D, K, L, T=ROOM_T):
    """True where the degree L meets the rule of truncation_degree (ceil(sigma) + 4 <= L)."""
    return np.ceil(anisotropy_ratio(D, K, T)) + 4 <= np.asarray(L)


def anisotropy_ratio(D, K, T=ROOM_T):
    """sigma = K V / (k_B T) with V = pi D^3 / 6."""
    return np.asarray(K) * (np.pi * np.asarray(D) ** 3 / 6) / (1.380649e-23 * T)


def lissajous_stratified_ids():
    """64 instances of the 2312-instance Lissajous batch: for every easy-axis angle j, the four corners
    and the centre of the 17 x 17 offset grid and three of the four edge midpoints (the edge left out
    turns with j).  Instance id = (j * 17 + iy) * 17 + ix."""
    ids = []
    mids = [(0, 8), (8, 16), (16, 8), (8, 0)]
    for j in range(8):
        pos = [(0, 0), (0, 16), (16, 0), (16, 16), (8, 8)] + [m for e, m in enumerate(mids) if e != j % 4]
        ids += [(j * 17 + iy) * 17 + ix for iy, ix in pos]
    return ids


def uneven_sweep(n=4096, seed=3, L_max=24):
    """Batched uneven sweep: D ~ U[15, 30] nm, K log-uniform in [0.5, 20] kJ/m^3, alpha ~ U[0.05, 0.3],
    easy axes uniform on the sphere, offsets U[-12, 12] mT in x and y, L by truncation_degree.
    Every draw is kept: about 12 % of the (D, K) pairs have sigma > 20, which no degree up to 24
    resolves (``resolvable`` tells them apart); the solver is expected to flag them, not to hide them."""
    r = np.random.default_rng(seed)
    D = r.uniform(15e-9, 30e-9, n)
    K = np.exp(r.uniform(np.log(500.0), np.log(2e4), n))
    alpha = r.uniform(0.05, 0.3, n)
    z = r.uniform(-1, 1, n)
    ph = r.uniform(0, 2 * np.pi, n)
    s = np.sqrt(1 - z * z)
    easy = np.stack([s * np.cos(ph), s * np.sin(ph), z], 1)
    off = np.stack([r.uniform(-12e-3, 12e-3, n), r.uniform(-12e-3, 12e-3, n), np.zeros(n)], 1)
    L = truncation_degree(D, K, hi=L_max)
    inst = _instances(D, np.full(n, MAGNETITE_MS), K, alpha, np.full(n, ROOM_T), easy, off, L)
    return dict(name=f"uneven_{n}_seed{seed}", inst=inst, drive=lissajous_drive(), samples=1632, settle=1,
                n_harm=200, harm_z=False)


def _particles_resolved_by(n, r, L_max, sigma_bias=0.0):
    """n draws of (D, K, alpha) from the uneven sweep's distribution, kept where truncation_degree <= L_max;
    with sigma_bias b > 0 a draw is also kept only with probability (1 + b sigma / sigma_max) / (1 + b)
    (sigma_max = L_max - 4), which moves weight toward the stiff end."""
    D, K, alpha = np.empty(0), np.empty(0), np.empty(0)
    while D.size < n:
        m = (4 if sigma_bias > 0 else 2) * (n - D.size) + 64
        d = r.uniform(15e-9, 30e-9, m)
        k = np.exp(r.uniform(np.log(500.0), np.log(2e4), m))
        a = r.uniform(0.05, 0.3, m)
        keep = truncation_degree(d, k) <= L_max
        if sigma_bias > 0:
            w = (1.0 + sigma_bias * anisotropy_ratio(d, k) / (L_max - 4)) / (1.0 + sigma_bias)
            keep &= r.uniform(0, 1, m) < w
        D, K, alpha = np.r_[D, d[keep]], np.r_[K, k[keep]], np.r_[alpha, a[keep]]
    return D[:n], K[:n], alpha[:n]


def fibonacci_axes(n):
    """n unit vectors of the Fibonacci lattice on the sphere (z = 1 - (2i + 1)/n, golden-angle azimuths)."""
    i = np.arange(n)
    z = 1.0 - (2 * i + 1) / n
    ph = i * np.pi * (3.0 - np.sqrt(5.0))
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], 1)


def surrogate_particles(n, seed, L_max=16, sigma_bias=0.0):
    """Training / held-out draws of the particle-family surrogate: (D, K, alpha) as in uneven_sweep but
    only particles that a degree <= L_max resolves, easy axes uniform on the sphere, offsets
    U[-12, 12] mT in x and y, L by truncation_degree (8..L_max); Lissajous drive, 1632 samples.
    sigma_bias > 0 (training sets only) draws the stiff particles more often (_particles_resolved_by)."""
    r = np.random.default_rng(seed)
    D, K, alpha = _particles_resolved_by(n, r, L_max, sigma_bias)
    z = r.uniform(-1, 1, n)
    ph = r.uniform(0, 2 * np.pi, n)
    s = np.sqrt(1 - z * z)
    easy = np.stack([s * np.cos(ph), s * np.sin(ph), z], 1)
    off = np.stack([r.uniform(-12e-3, 12e-3, n), r.uniform(-12e-3, 12e-3, n), np.zeros(n)], 1)
    inst = _instances(D, np.full(n, MAGNETITE_MS), K, alpha, np.full(n, ROOM_T), easy, off,
                      truncation_degree(D, K, hi=L_max))
    return dict(inst=inst, drive=lissajous_drive(), samples=1632, settle=1)


def surrogate_particle_grid(n_sets=8, n_axes=64, n_off=64, seed=50, L_max=16):
    """Evaluation grid of the particle-family surrogate: n_sets (D, K, alpha) drawn like
    surrogate_particles, each on n_axes Fibonacci axes x an n_off x n_off grid of offsets on +-12 mT
    (instance order: set, axis, offset y, offset x)."""
    r = np.random.default_rng(seed)
    D, K, alpha = _particles_resolved_by(n_sets, r, L_max)
    g = -12e-3 + 24e-3 * (np.arange(n_off) + 0.5) / n_off
    p, a, iy, ix = np.meshgrid(np.arange(n_sets), np.arange(n_axes), np.arange(n_off), np.arange(n_off),
                               indexing="ij")
    p, a, iy, ix = p.ravel(), a.ravel(), iy.ravel(), ix.ravel()
    n = p.size
    off = np.stack([g[ix], g[iy], np.zeros(n)], 1)
    inst = _instances(D[p], np.full(n, MAGNETITE_MS), K[p], alpha[p], np.full(n, ROOM_T), fibonacci_axes(n_axes)[a],
                      off, truncation_degree(D[p], K[p], hi=L_max))
    return dict(inst=inst, drive=lissajous_drive(), samples=1632, settle=1)


def identification_problem(n_off=32, n_ang=16, n_comp=4, L=16, span=12e-3, n_harm=300, seed=4, noise_seed=40):
    """Parameter identification by gradient (the adjoint workload): an n_off x n_off grid of offsets on
    +-span (endpoints included) x n_ang in-plane easy-axis angles j pi / n_ang (from x) x n_comp particle
    components, each with its own D, K, alpha and superposition weight; L fixed, the Lissajous drive,
    harmonics 1..n_harm of x and y.  Ground truth (seed): D ~ U[16, 28] nm, K log-uniform in
    [0.5, 5] kJ/m^3, alpha ~ U[0.05, 0.3], w ~ U[0.1, 1].  The gradient is taken at a fixed guess away
    from the truth (D x 1.05, K x 1.1, alpha x 0.9, w x 0.95, angles + 0.02 rad).  The measured signal is
    the truth's superposition plus Gaussian noise (noise_seed) of 1 % of each channel's RMS, drawn by
    the consumer with noise_rng() since it needs the clean signal."""
    r = np.random.default_rng(seed)
    truth = dict(D=r.uniform(16e-9, 28e-9, n_comp), K=np.exp(r.uniform(np.log(500.0), np.log(5e3), n_comp)),
                 alpha=r.uniform(0.05, 0.3, n_comp), w=r.uniform(0.1, 1.0, n_comp))
    guess = dict(D=truth["D"] * 1.05, K=truth["K"] * 1.1, alpha=truth["alpha"] * 0.9, w=truth["w"] * 0.95)
    g = -span + (2 * span / (n_off - 1)) * np.arange(n_off)
    iy, ix = np.meshgrid(np.arange(n_off), np.arange(n_off), indexing="ij")
    off = np.stack([g[ix.ravel()], g[iy.ravel()], np.zeros(n_off * n_off)], 1)
    angles = np.arange(n_ang) * np.pi / n_ang
    return dict(name=f"identification_{n_off}x{n_off}x{n_ang}x{n_comp}_L{L}", offsets=off, angles=angles,
                angles_guess=angles + 0.02, truth=truth, guess=guess, Ms=MAGNETITE_MS, T=ROOM_T, L=L,
                drive=lissajous_drive(), samples=1632, settle=1, n_harm=n_harm, noise_frac=0.01,
                noise_rng=lambda: np.random.default_rng(noise_seed))


def identification_instances(ws, angle_index, which="guess"):
    """The instances of one easy-axis angle of an identification problem as an instance set
    (instance = offset index * n_comp + component), with the guess or the truth parameters."""
    p = ws[which]
    nC = p["D"].size
    nO = ws["offsets"].shape[0]
    a = (ws["angles_guess"] if which == "guess" else ws["angles"])[angle_index]
    n = nO * nC
    inst = _instances(np.tile(p["D"], nO), np.full(n, ws["Ms"]), np.tile(p["K"], nO), np.tile(p["alpha"], nO),
                      np.full(n, ws["T"]), np.tile([np.cos(a), np.sin(a), 0.0], (n, 1)),
                      np.repeat(ws["offsets"], nC, 0), np.full(n, ws["L"]))
    return dict(name=f"{ws['name']}_{which}_angle{angle_index}", inst=inst, drive=ws["drive"], samples=ws["samples"],
                settle=ws["settle"], n_harm=ws["n_harm"], harm_z=False)


def small_random(n, L, seed, samples=64, settle=1, n_harm=10, freq_scale=1.0, resolved=True):
    """Small random instances for parity tests (short synthetic drive with 3 and 4 cycles per period).
    resolved: particles that the degree L does not resolve (``resolvable`` False, i.e. sigma > L - 4)
    get (D, K) drawn again from a second generator (seeded by (seed, 1)) after all other draws, so a
    seed without such particles gives the same instances either way.  Below L = 5 no particle of the
    range meets the rule and nothing is redrawn."""
    r = np.random.default_rng(seed)
    D = r.uniform(14e-9, 24e-9, n)
    K = np.exp(r.uniform(np.log(300.0), np.log(8e3), n))
    alpha = r.uniform(0.05, 0.3, n)
    v = r.normal(size=(n, 3))
    easy = v / np.linalg.norm(v, axis=1, keepdims=True)
    off = r.uniform(-6e-3, 6e-3, (n, 3))
    if resolved and L >= 5:
        r2 = np.random.default_rng([seed, 1])
        while True:
            bad = np.nonzero(~resolvable(D, K, np.full(n, L)))[0]
            if bad.size == 0:
                break
            D[bad] = r2.uniform(14e-9, 24e-9, bad.size)
            K[bad] = np.exp(r2.uniform(np.log(300.0), np.log(8e3), bad.size))
    inst = _instances(D, np.full(n, MAGNETITE_MS), K, alpha, np.full(n, ROOM_T), easy, off, np.full(n, L))
    T = 40e-6 / freq_scale
    drive = dict(amp=(10e-3, 8e-3, 3e-3), freq=(3 / T, 4 / T, 1 / T), phase=(0.0, 0.3, -0.7), period=T)
    return dict(name=f"small_L{L}_seed{seed}", inst=inst, drive=drive, samples=samples, settle=settle,
                n_harm=n_harm, harm_z=True)


def fv_crosscheck(n=6, seed=61):
    """Instances for the finite-volume cross-check of the truncation in L: a fast drive (period 4 us,
    components at 0.75 / 1 / 0.25 MHz, 10 / 8 / 3 mT) where the precession term moves the response by
    about 1 %, 64 samples, one settling period; D ~ U[16, 21] nm, K log-uniform in [0.5, 6] kJ/m^3
    (sigma up to about 7),
    alpha ~ U[0.05, 0.2], easy axes uniform on the sphere, offsets U[-3, 3] mT, L by
    truncation_degree."""
    r = np.random.default_rng(seed)
    D = r.uniform(16e-9, 21e-9, n)
    K = np.exp(r.uniform(np.log(500.0), np.log(6e3), n))
    alpha = r.uniform(0.05, 0.2, n)
    v = r.normal(size=(n, 3))
    easy = v / np.linalg.norm(v, axis=1, keepdims=True)
    off = r.uniform(-3e-3, 3e-3, (n, 3))
    inst = _instances(D, np.full(n, MAGNETITE_MS), K, alpha, np.full(n, ROOM_T), easy, off,
                      truncation_degree(D, K))
    T = 4e-6
    drive = dict(amp=(10e-3, 8e-3, 3e-3), freq=(3 / T, 4 / T, 1 / T), phase=(0.0, 0.3, -0.7), period=T)
    return dict(name="fv_crosscheck", inst=inst, drive=drive, samples=64, settle=1, n_harm=10, harm_z=True)


def take(ws, idx):
    """Sub-workload with the instances at `idx`."""
    idx = np.asarray(idx, dtype=np.int64)
    out = dict(ws)
    out["inst"] = {k: v[idx] for k, v in ws["inst"].items()}
    return out


def random_system_matrices(n, n_pos, n_ch, n_bins, seed):
    """n complex64 system matrices [n, n_pos, n_ch, n_bins] with standard normal real and imaginary
    parts (inputs of the fit and distance-measure parity tests)."""
    r = np.random.default_rng(seed)
    x = r.normal(size=(n, n_pos, n_ch, n_bins)) + 1j * r.normal(size=(n, n_pos, n_ch, n_bins))
    return x.astype(np.complex64)


M1_DRIVE_AMP = (12.59e-3, 13.55e-3, 0.0)   # the paper's calibrated drive amplitudes (mu0 H, T)
M1_SPAN = (14.35e-3, 14.71e-3)             # half-widths of its 11 x 11 offset grid (mu0 H, T)


def m1_dictionary(D_set, K_set, angles_deg, n_grid=11, samples=1632, n_harm=200, L_max=24):
    """Dictionary of model M1 (Simulation Setting): every (D, K, angle) of the given sets at every offset
    of an n_grid x n_grid grid spanning the paper's offset ranges, with the paper's Lissajous drive.
    Instances are ordered element-major ((D, K, angle), angle fastest), offset position minor
    (x fastest), so fpn_solve's harmonics are directly the dictionary layout of fpn_fit_rows.  The
    degree of each instance follows ``truncation_degree``; easy axes in the xy-plane at the angle
    from x (the same convention as the other workloads)."""
    gx = np.linspace(-M1_SPAN[0], M1_SPAN[0], n_grid)
    gy = np.linspace(-M1_SPAN[1], M1_SPAN[1], n_grid)
    offs = np.array([(x, y, 0.0) for y in gy for x in gx])
    rows = [(D, K, a) for D in D_set for K in K_set for a in angles_deg]
    n_el, n_pos = len(rows), len(offs)
    D = np.repeat([r[0] for r in rows], n_pos)
    K = np.repeat([r[1] for r in rows], n_pos)
    th = np.deg2rad(np.repeat([r[2] for r in rows], n_pos))
    easy = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], 1)
    off = np.tile(offs, (n_el, 1))
    n = n_el * n_pos
    L = truncation_degree(D, K, hi=L_max)
    inst = _instances(D, np.full(n, MAGNETITE_MS), K, np.full(n, 0.1), np.full(n, ROOM_T), easy, off, L)
    drive = dict(amp=M1_DRIVE_AMP, freq=LISSAJOUS_F, phase=(0.0, 0.0, 0.0), period=LISSAJOUS_T)
    return dict(name=f"m1_dictionary_{len(D_set)}x{len(K_set)}x{len(angles_deg)}_{n_grid}x{n_grid}", inst=inst,
                drive=drive, samples=samples, settle=1, n_harm=n_harm, harm_z=False, n_elements=n_el,
                n_pos=n_pos, elements=rows)


def m1_transfer_and_noise(n_ang, n_pos, n_ch, n_bins, seed, rel_noise=0.01):
    """Synthetic receive chain for the M1 demonstration: a complex transfer value per (channel, bin)
    (log-normal magnitude, uniform phase) and unit complex Gaussian noise [n_ang, n_pos, n_ch, n_bins];
    the caller scales the noise by rel_noise times each row's RMS."""
    r = np.random.default_rng(seed)
    a = np.exp(r.normal(0.0, 0.3, (n_ch, n_bins))) * np.exp(1j * r.uniform(-np.pi, np.pi, (n_ch, n_bins)))
    z = (r.normal(size=(n_ang, n_pos, n_ch, n_bins)) + 1j * r.normal(size=(n_ang, n_pos, n_ch, n_bins))) / np.sqrt(2)
    return a, z, rel_noise
