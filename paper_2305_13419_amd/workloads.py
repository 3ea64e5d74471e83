"""Seeded synthetic inputs shaped like the paper's workloads.

Input generation only: grids, spacings, time steps, per-cell material maps,
initial fields, source and probe placements.  Nothing here evaluates the
scheme; the same arrays are fed to the HIP path and to the CPU oracle.

Every workload is a plain dict:
  shape (nx, ny, nz), spacing (dx, dy, dz), dt, theta, pml (per axis None or
  (lo, hi)), maps (eps_r, sigma, inv_lambda2) as float64 arrays (nz, ny, nx),
  fields (E, H, J) at t = 0 as lists of float64 arrays or None (all zero),
  sources and probes as lists of dicts, steps.
"""
import numpy as np

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
C0 = 1.0 / np.sqrt(EPS0 * MU0)


def courant_dt(spacing, inv_lambda2_max, fraction):
    """fraction x the largest stable dt of the scheme with a London term (eps_r >= 1):
    2 / (c0 sqrt(sum 4/d^2 + max 1/lambda^2))."""
    s = sum(4.0 / (d * d) for d in spacing)
    return fraction * 2.0 / (C0 * np.sqrt(s + inv_lambda2_max))


def random_boxes(shape, rng, fill=0.30, side=(4, 32), lam=(50e-9, 200e-9), sig=(1e3, 1e5),
                 eps_r=None):
    """Random axis-aligned superconducting boxes (integer sides uniform in `side`, uniform wrapped
    positions, lambda_L and sigma_n linear-uniform), painted in order until `fill` of the cells are
    superconducting.  Returns float64 maps (eps_r, sigma, inv_lambda2) of shape (nz, ny, nx)."""
    nx, ny, nz = shape
    ell = np.zeros((nz, ny, nx))
    sg = np.zeros((nz, ny, nx))
    er = np.ones((nz, ny, nx)) if eps_r is None else np.array(eps_r, dtype=np.float64, copy=True)
    target = fill * nx * ny * nz
    count = 0
    while count < target:
        w = rng.integers(side[0], side[1] + 1, size=3)
        o = np.array([rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)])
        lam_b = rng.uniform(*lam)
        sig_b = rng.uniform(*sig)
        ix = (o[0] + np.arange(min(w[0], nx))) % nx
        iy = (o[1] + np.arange(min(w[1], ny))) % ny
        iz = (o[2] + np.arange(min(w[2], nz))) % nz
        sel = np.ix_(iz, iy, ix)
        before = np.count_nonzero(ell[sel])
        ell[sel] = 1.0 / lam_b**2
        sg[sel] = sig_b
        er[sel] = 1.0
        count += ell[sel].size - before
    return er, sg, ell


def roofline_grid(n=256, seed=2, d=20e-9, steps=1000):
    """Roofline workload: n^3 cells, dx = 20 nm, periodic on all sides, random superconducting boxes
    (lambda_L in 50-200 nm, sigma_n in 1e3-1e5 S/m) filling ~30 % of the cells, eps_r = 1, E and H
    drawn from N(0, 1), Js = 0, theta = 1, dt = 0.95 x the stable limit for lambda_L >= 50 nm."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    maps = random_boxes(shape, rng)
    nz, ny, nx = shape[2], shape[1], shape[0]
    E = [rng.standard_normal((nz, ny, nx)) for _ in range(3)]
    H = [rng.standard_normal((nz, ny, nx)) for _ in range(3)]
    return dict(name=f"roofline {shape[0]}x{shape[1]}x{shape[2]}", shape=shape, spacing=(d, d, d),
                dt=courant_dt((d, d, d), 1.0 / (50e-9) ** 2, 0.95), theta=1.0, pml=(None, None, None),
                maps=maps, fields=(E, H, None), sources=[], probes=[], steps=steps)


def skin_depth_grid(sc=True, steps=26225, ny=4, nz=4):
    """Skin-depth / reflection workload: 512 x 4 x 4 cells of 10 nm, periodic in y and z, CPML of 32
    cells at both x ends; vacuum for x < 256 and a superconductor (lambda_L = 100 nm, sigma_n = 1e4
    S/m, eps_r = 1) for x >= 256 (sc=False: all vacuum, the reference run); a soft 10 THz sine Ey
    source of 1 V/m on node plane x = 64; dt = 0.99 dx / (c sqrt 3); theta = 1."""
    nx, d = 512, 10e-9
    shp = (nz, ny, nx)
    ell = np.zeros(shp)
    sig = np.zeros(shp)
    if sc:
        ell[..., 256:] = 1e14
        sig[..., 256:] = 1e4
    f = 10e12
    return dict(name="skin depth 512x4x4", shape=(nx, ny, nz), spacing=(d, d, d),
                dt=0.99 * d / (C0 * np.sqrt(3.0)), theta=1.0, pml=((32, 32), None, None),
                maps=(np.ones(shp), sig, ell), fields=None,
                sources=[dict(comp=1, box=(64, 65, 0, ny, 0, nz), amplitude=1.0, waveform="sin", freq=f)],
                probes=[dict(comp=1, box=(160, 161, 0, ny, 0, nz), freqs=(f,))],
                freq=f, steps=steps)


def random_medium(shape, seed, pml=(None, None, None), d=(20e-9, 17e-9, 23e-9), theta=1.0, fill=0.4,
                  field_scale=1.0, sigma_max=1e5):
    """Small heterogeneous test medium: per-cell random eps_r in [1, 4], sigma_n in [0, sigma_max] on
    half of the cells, superconducting cells (lambda_L 50-200 nm) on a `fill` fraction; random fields."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    shp = (nz, ny, nx)
    ell = np.where(rng.random(shp) < fill, 1.0 / rng.uniform(50e-9, 200e-9, shp) ** 2, 0.0)
    eps = rng.uniform(1.0, 4.0, shp)
    sig = np.where(rng.random(shp) < 0.5, rng.uniform(0.0, sigma_max, shp), 0.0)
    E = [field_scale * rng.standard_normal(shp) for _ in range(3)]
    H = [field_scale * rng.standard_normal(shp) / 377.0 for _ in range(3)]
    J = [np.where(ell > 0, 1e3 * rng.standard_normal(shp), 0.0) for _ in range(3)]
    return dict(name=f"random medium {nx}x{ny}x{nz}", shape=shape, spacing=tuple(d),
                dt=courant_dt(d, 1.0 / (50e-9) ** 2, 0.95), theta=theta, pml=pml,
                maps=(eps, sig, ell), fields=(E, H, J), sources=[], probes=[], steps=20)


def cpw_grid(scale=1, steps=None, dtype_note="FP32 fields + FP64 probes"):
    """Coplanar-waveguide resonator shaped like the paper's device (Sec. 5), at reduced size.

    scale=1: 512 x 256 x 128 cells of 0.5 um; scale=2 halves every length (256 x 128 x 64), scale=4
    quarters it (128 x 64 x 32, the film one cell thick: the generator at a size the oracle steps 20 000
    times in about a minute).
    eps_r = 11.7 substrate below the film; a 4-cell (2 at scale 2) superconducting film
    (lambda_L = 100 nm, sigma_n = 1e4 S/m) patterned as a centre strip with two gaps and ground
    planes reaching the periodic y edges; the strip is cut by two coupling gaps into input port,
    half-wave resonator and output port; the pattern stops one PML width short of the x-PML.
    CPML on the x and z faces.  Excitation: opposite soft Ey Gaussian-modulated pulses in the two
    gaps near the input end (f = 0.96 THz x scale; tw = 1/(2f), t0 = 4 tw).
    dt = 0.95 x the stable limit with the London term."""
    s = scale
    nx, ny, nz = 512 // s, 256 // s, 128 // s
    d = 0.5e-6
    npml = 16 // s
    k_film0, k_film1 = 48 // s, 52 // s
    strip = (118 // s, 138 // s)
    gap_lo = (106 // s, strip[0])
    gap_hi = (strip[1], 150 // s)
    x0, x1 = 32 // s, 480 // s
    cg1 = (190 // s, 194 // s)
    cg2 = (318 // s, 322 // s)
    shp = (nz, ny, nx)
    eps = np.ones(shp)
    eps[:k_film0] = 11.7
    film = np.zeros((ny, nx), bool)
    film[:, x0:x1] = True                       # ground planes and strip region
    film[gap_lo[0]:gap_lo[1], x0:x1] = False    # the two gaps
    film[gap_hi[0]:gap_hi[1], x0:x1] = False
    film[strip[0]:strip[1], cg1[0]:cg1[1]] = False  # coupling gaps cut the strip
    film[strip[0]:strip[1], cg2[0]:cg2[1]] = False
    ell = np.zeros(shp)
    sig = np.zeros(shp)
    ell[k_film0:k_film1][:, film] = 1e14
    sig[k_film0:k_film1][:, film] = 1e4
    f = 0.96e12 * s
    tw = 1.0 / (2 * f)
    xs = 40 // s
    kk = (k_film0, k_film1 + 1)
    src = [dict(comp=1, box=(xs, xs + 1, gap_lo[0], gap_lo[1], kk[0], kk[1]), amplitude=1.0, waveform="mod_gauss",
                freq=f, t0=4 * tw, tw=tw),
           dict(comp=1, box=(xs, xs + 1, gap_hi[0], gap_hi[1], kk[0], kk[1]), amplitude=-1.0, waveform="mod_gauss",
                freq=f, t0=4 * tw, tw=tw)]
    xp = cg1[1] + 4 // s
    kmid = (k_film0 + k_film1) // 2
    probes = [dict(comp=1, box=(xp, xp + 1, gap_lo[0] + 6 // s, gap_lo[0] + 6 // s + 1, kmid, kmid + 1)),
              dict(comp=1, box=(xp, xp + 1, gap_lo[0], gap_lo[1], kmid, kmid + 1))]
    return dict(name=f"cpw {nx}x{ny}x{nz}", shape=(nx, ny, nz), spacing=(d, d, d),
                dt=courant_dt((d, d, d), 1e14, 0.95), theta=1.0, pml=((npml, npml), None, (npml, npml)),
                maps=(eps, sig, ell), fields=None, sources=src, probes=probes, freq=f,
                steps=steps if steps is not None else (20000 if s == 1 else 4096),
                # objective frequency at scale 2: the peak of |DFT| of the gap line in an unperturbed FP64
                # run (1.7453 THz), frozen as a constant for every gradient and finite-difference run
                objective=(1, probes[1]["box"], 1.7453e12 if s == 2 else None), note=dtype_note)


def large_mixed_grid(seed=5, steps=8192, shape=(1024, 512, 256)):
    """Large mixed-precision workload: 1024 x 512 x 256 cells of 20 nm, periodic, eps_r = 11.7 in the
    bottom quarter, random superconducting boxes as in the roofline grid (seed 5), zero fields driven by
    a soft Ey sheet source at x = nx/4 over the middle quarter of z; objective: Ey summed along y at
    x = nx/2, z = nz/2.  `shape` gives the same construction on another grid (parity tests at the
    full step count on a grid the oracle can step)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in shape)
    eps0 = np.ones((nz, ny, nx))
    eps0[:nz // 4] = 11.7
    maps = random_boxes((nx, ny, nz), rng, eps_r=eps0)
    d = 20e-9
    f = 2e14
    tw = 1.0 / (2 * f)
    obj_box = (nx // 2, nx // 2 + 1, 0, ny, nz // 2, nz // 2 + 1)
    return dict(name=f"large {nx}x{ny}x{nz}", shape=(nx, ny, nz), spacing=(d, d, d),
                dt=courant_dt((d, d, d), 1.0 / (50e-9) ** 2, 0.95), theta=1.0, pml=(None, None, None),
                maps=maps, fields=None,
                sources=[dict(comp=1, box=(nx // 4, nx // 4 + 1, 0, ny, 3 * nz // 8, 5 * nz // 8), amplitude=1.0,
                              waveform="mod_gauss", freq=f, t0=4 * tw, tw=tw)],
                probes=[dict(comp=1, box=obj_box)], freq=f, steps=steps,
                objective=(1, obj_box, None))


# Rows of the paper's skin-depth sweep (Sec. 4.1, Table 1): (sigma S/m, f Hz, paper's computed delta nm).
TABLE1_ROWS = [(0.0, 25e9, 400), (0.0, 100e9, 400), (0.0, 1e12, 400), (0.0, 1e14, 739),
               (1e4, 25e9, 400), (1e4, 100e9, 400), (1e4, 1e12, 400), (1e4, 1e14, 450),
               (1e7, 25e9, 395), (1e7, 100e9, 350), (1e7, 1e12, 153), (1e7, 1e14, 13)]


def table1_grid(sigma, freq, delta_theory, half=3000, npml=32, periods=5):
    """One row of the skin-depth sweep: a homogeneous superconductor (lambda_L = 400 nm, eps_r = 1,
    sigma_n = sigma) on a 1-D line of 10 nm cells along x (ny = nz = 1; dy = dz = 1 m so the stability
    bound is the 1-D one), dt = 0.03 fs, a soft Ey sine of frequency freq on the centre node, run to 5
    periods (the paper's run) unless `periods` says otherwise.  The paper's domains (+-32 um .. +-128 mm) only keep the start-up transient away from the
    ends; here `half` cells on each side (30 um, > 40 skin depths) end in CPML slabs that absorb it.
    Probes: Ey at the source node and at the node nearest to delta_theory from it (the paper's z0)."""
    d = 10e-9
    nx = 2 * half + 2 * npml + 1
    shp = (1, 1, nx)
    ic = nx // 2
    z0 = max(1, int(round(delta_theory / d)))
    dt = 3e-17
    steps = int(np.ceil(periods / freq / dt))
    return dict(name=f"table1 sigma={sigma:g} f={freq:g}", shape=(nx, 1, 1), spacing=(d, 1.0, 1.0), dt=dt,
                theta=1.0, pml=((npml, npml), None, None),
                maps=(np.ones(shp), np.full(shp, float(sigma)), np.full(shp, 1.0 / (400e-9) ** 2)),
                fields=None,
                sources=[dict(comp=1, box=(ic, ic + 1, 0, 1, 0, 1), amplitude=1.0, waveform="sin", freq=freq)],
                probes=[dict(comp=1, box=(ic, ic + 1, 0, 1, 0, 1)), dict(comp=1, box=(ic + z0, ic + z0 + 1, 0, 1, 0, 1))],
                z0=z0 * d, freq=freq, steps=steps)


def steady_amplitude(series, dt, freq, periods=2):
    """Amplitude of the steady oscillation at freq: least-squares fit of a cos + b sin + c over the last
    `periods` periods of the series (sample n at time n dt)."""
    series = np.asarray(series, dtype=np.float64)
    m = int(round(periods / freq / dt))
    t = np.arange(series.size - m, series.size) * dt
    A = np.stack([np.cos(2 * np.pi * freq * t), np.sin(2 * np.pi * freq * t), np.ones_like(t)], axis=1)
    coef, *_ = np.linalg.lstsq(A, series[-m:], rcond=None)
    return float(np.hypot(coef[0], coef[1]))


# Material of the film in the four cases of the paper's CPW study (Sec. 5, Table 7): (sigma S/m,
# 1/lambda_L^2 m^-2) and the paper's Q and computed resonance (GHz).
PAPER_CPW_CASES = {1: (6e7, 0.0, 24, 96.9), 2: (1e10, 0.0, 491, 98.2), 3: (6e7, 1e14, 316, 97.1),
                   4: (0.0, 1e14, 973, 97.1)}


def paper_cpw_grid(case=3, npml=(8, 8, 16), fields=None, seed=11, dz=50e-9, dt=None, film_sigma=None):
    """The paper's coplanar-waveguide resonator at its own size (Sec. 5): the domain [-65, 65] um x
    [-504, 504] um x [0, 64] um in 130 x 1008 x 1280 cells (dx = dy = 1 um, dz = 50 nm), with CPML
    slabs of npml cells added outside it on every face (the paper's PML is outside its domain too).
    Silicon substrate (eps_r = 11.7) for z < 32 um, a 200 nm film on it patterned as two ground planes
    (50 um wide, 1000 um long), two 6 um gaps and the 10 um centre line cut along y into input port
    [-500, -400] um, coupling gap, resonator [-300, 300] um, coupling gap, output port [400, 500] um;
    vacuum above; the film material is that of `case` (PAPER_CPW_CASES).  Source: opposite soft Ex
    Gaussian-modulated sines exp(-(t - 4T)^2 / (2 T^2)) sin(2 pi t / T), T = 1 / 100 GHz, in the two gaps
    at y = -500 um over the film thickness.  Probes: Ex in the left gap at y = -450 um and -300 um, on
    the film's middle plane.  dt defaults to 0.95 x the stable limit with the London term (0.158 fs,
    the paper's).  fields='random' gives seeded N(0, 1) initial fields (parity tests).  film_sigma
    replaces the case's film conductivity (the Q runs' sensitivity study)."""
    sig_f, ell_f, _, _ = PAPER_CPW_CASES[case]
    if film_sigma is not None:
        sig_f = float(film_sigma)
    px, py, pz = npml
    dx = dy = 1e-6
    nx, ny, nz = 130 + 2 * px, 1008 + 2 * py, int(round(64e-6 / dz)) + 2 * pz
    shp = (nz, ny, nx)
    # cell centres in um (x, y) and nm-free z index of the domain
    xc = (np.arange(nx) - px) * 1.0 - 65.0 + 0.5
    yc = (np.arange(ny) - py) * 1.0 - 504.0 + 0.5
    kz = np.arange(nz) - pz                         # cell k spans [kz dz, (kz + 1) dz]
    k_sub = int(round(32e-6 / dz))                  # substrate cells kz < k_sub
    k_film = k_sub + int(round(200e-9 / dz))        # film cells k_sub <= kz < k_film
    eps = np.ones(shp)
    eps[kz < k_sub] = 11.7
    X, Y = np.meshgrid(xc, yc)                      # (ny, nx)
    inside_y = np.abs(Y) < 500.0
    ground = inside_y & (np.abs(X) > 11.0) & (np.abs(X) < 61.0)
    line = (np.abs(X) < 5.0) & (((Y > -500.0) & (Y < -400.0)) | ((Y > -300.0) & (Y < 300.0)) |
                                ((Y > 400.0) & (Y < 500.0)))
    film = ground | line
    sig = np.zeros(shp)
    ell = np.zeros(shp)
    fz = (kz >= k_sub) & (kz < k_film)
    sig[np.ix_(fz, np.ones(ny, bool), np.ones(nx, bool))] = np.where(film, sig_f, 0.0)[None]
    ell[np.ix_(fz, np.ones(ny, bool), np.ones(nx, bool))] = np.where(film, ell_f, 0.0)[None]
    if dt is None:
        dt = courant_dt((dx, dy, dz), 1e14, 0.95)
    f = 100e9
    T = 1.0 / f
    i_of = lambda x: int(np.floor(x + 65.0)) + px    # noqa: E731  (cell index holding coordinate x um)
    j_of = lambda y: int(np.floor(y + 504.0)) + py   # noqa: E731
    k0, k1 = k_sub + pz, k_film + pz + 1             # Ex edges on the film's node planes
    js = j_of(-500.0)
    src = [dict(comp=0, box=(i_of(-11.0), i_of(-5.0), js, js + 1, k0, k1), amplitude=1.0, waveform="mod_gauss",
                freq=f, t0=4 * T, tw=T),
           dict(comp=0, box=(i_of(5.0), i_of(11.0), js, js + 1, k0, k1), amplitude=-1.0, waveform="mod_gauss",
                freq=f, t0=4 * T, tw=T)]
    km = (k_sub + k_film) // 2 + pz
    probes = [dict(comp=0, box=(i_of(-8.0), i_of(-8.0) + 1, j_of(-450.0), j_of(-450.0) + 1, km, km + 1)),
              dict(comp=0, box=(i_of(-8.0), i_of(-8.0) + 1, j_of(-300.0), j_of(-300.0) + 1, km, km + 1))]
    F = None
    if fields == "random":
        rng = np.random.default_rng(seed)
        E = [rng.standard_normal(shp) for _ in range(3)]
        H = [rng.standard_normal(shp) / 377.0 for _ in range(3)]
        F = (E, H, None)
    return dict(name=f"paper cpw {nx}x{ny}x{nz} case {case}", shape=(nx, ny, nz), spacing=(dx, dy, dz), dt=dt,
                theta=1.0, pml=((px, px), (py, py), (pz, pz)), maps=(eps, sig, ell), fields=F, sources=src,
                probes=probes, freq=f, steps=850000)
