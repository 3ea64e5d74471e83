"""The paper's convergence studies (Sec. 4.3, Tables 2-6) on the HIP path at the paper's sizes.  Tables
5 and 6 (Sec. 4.3.3): a cube of superconductor (lambda_L = 40 nm, sigma_n = 1e4 S/m, the paper's case (d)) from
-40 to 40 nm in a periodic vacuum domain [-640, 640] nm^3, hit by the plane Gaussian pulse
Ex = exp(-(z - z0)^2 / L^2), By = Ex / c (z0 = -320 nm, L = 80 nm), theta = 0.5 (the scheme's
second-order form, as for Tables 2-4), to t = 1.73 fs.

Time (Table 5): 256^3 cells, CFL 0.9 / 0.45 / 0.225 (200 / 400 / 800 steps).  Space (Table 6):
128^3 / 256^3 / 512^3 cells with the time step of 512^3 at CFL 0.9, 400 steps.  Errors are L1 means of
the difference between consecutive resolutions; for space, the finer solution is first restricted to
the coarser grid: along an axis where a component sits on nodes the coincident fine sample is taken,
along an axis where it sits on half nodes the two fine samples around the coarse one are averaged (so
an E edge is the mean of the 2 fine edges that tile it, a B face the mean of the 4 fine faces).  The GPU
FP64 path equals the oracle to ~1e-13 on every parity test, so these runs reproduce the oracle's
tables at sizes the oracle cannot step in reasonable time.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
C0 = 1.0 / np.sqrt(EPS0 * MU0)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "convergence_tables.txt")
COMPS = ["Ex", "Ey", "Ez", "Bx", "By", "Bz"]
# array axes (z, y, x) along which each component sits on half nodes
HALF = {"Ex": (2,), "Ey": (1,), "Ez": (0,), "Bx": (0, 1), "By": (0, 2), "Bz": (1, 2)}


def tables():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t, fld, a, b, r = line.split()
            rows[(t, fld)] = (float(a), float(b), float(r))
    return rows


def cube_run(n, dt, steps, region="cube", zp=-320e-9):
    """Integer-time (Ex, Ey, Ez, Bx, By, Bz) on the device after `steps` steps on n^3 cells.  The
    superconductor fills the cube (Tables 5-6), the strip -40 < z < 40 nm over all x and y (Tables 3-4),
    the whole domain (Table 2), or, with "smooth", the half z > 0 with lambda_L falling smoothly from 400
    to 40 nm and sigma = 0 (Sec. 4.3.2); zp is the pulse's initial centre."""
    from paper_2305_13419_amd import Simulation
    d = 1280e-9 / n
    sim = Simulation((n, n, n), (d, d, d), dt, 0.5, torch.float64)
    dev = sim.device
    c = -640e-9 + (torch.arange(n, device=dev, dtype=torch.float64) + 0.5) * d  # cell centres
    inside = (c > -40e-9) & (c < 40e-9)
    every = torch.ones_like(inside)
    if region == "cube":
        sc = inside[:, None, None] & inside[None, :, None] & inside[None, None, :]
    elif region == "strip":
        sc = inside[:, None, None] & every[None, :, None] & every[None, None, :]
    else:
        sc = every[:, None, None] & every[None, :, None] & every[None, None, :]
    z0 = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    if region == "smooth":  # sigma = 0, lambda_L from 400 nm at z = 0 to 40 nm at the domain's end (z > 0 only)
        lam = 400e-9 + (40e-9 - 400e-9) * torch.clamp(c / 640e-9, 0.0, 1.0)
        ell = torch.where(c > 0, 1.0 / lam**2, 0.0)[:, None, None].expand(n, n, n).contiguous()
        sim.set_materials(torch.ones_like(z0), z0, ell)
        del ell
    else:
        sim.set_materials(torch.ones_like(z0), torch.where(sc, 1e4, 0.0), torch.where(sc, 1.0 / (40e-9) ** 2, 0.0))
    zn = -640e-9 + torch.arange(n, device=dev, dtype=torch.float64) * d  # z of node k
    L = 80e-9
    ex = torch.exp(-((zn - zp) ** 2) / L**2)[:, None, None].expand(n, n, n).contiguous()
    hy = (torch.exp(-((zn + d / 2 - zp) ** 2) / L**2) / (C0 * MU0))[:, None, None].expand(n, n, n).contiguous()
    sim.set_fields([ex, z0, z0], [z0, hy, z0], [z0, z0, z0])
    del ex, hy
    sim.step(steps)
    E, H, _ = sim.integer_time_fields()
    out = dict(zip(COMPS, list(E) + [h * MU0 for h in H]))
    sim.close()
    torch.cuda.empty_cache()
    return out


def restrict(F, comp):
    """Fine -> coarse: average the two fine samples along half-node axes, take every other sample
    along node axes."""
    for ax in range(3):
        a = F.narrow(ax, 0, F.shape[ax] // 2 * 2)
        even = a.index_select(ax, torch.arange(0, a.shape[ax], 2, device=a.device))
        if ax in HALF[comp]:
            odd = a.index_select(ax, torch.arange(1, a.shape[ax], 2, device=a.device))
            F = 0.5 * (even + odd)
        else:
            F = even
    return F


def l1(a, b):
    return float((a - b).abs().mean())


def test_table5_cube_time_convergence():
    ref = tables()
    dt09 = 0.9 * 5e-9 / (C0 * np.sqrt(3))
    sols = [cube_run(256, dt09 * f, st) for f, st in ((1.0, 200), (0.5, 400), (0.25, 800))]
    for comp in COMPS:
        e1 = l1(sols[1][comp], sols[0][comp])
        e2 = l1(sols[2][comp], sols[1][comp])
        rate = np.log2(e1 / e2)
        a, b, r = ref[("table5", comp)]
        print(f"Table 5 {comp}: {e1:.3e} {e2:.3e} rate {rate:.3f}  (paper {a:.3e} {b:.3e} {r:.2f})", flush=True)
        assert abs(rate - r) < 0.02
        assert abs(e1 / a - 1) < 0.10 and abs(e2 / b - 1) < 0.10


def test_table6_cube_space_convergence():
    ref = tables()
    dt = 0.9 * 2.5e-9 / (C0 * np.sqrt(3))
    errs = {c: [] for c in COMPS}
    prev = None
    for n in (128, 256, 512):
        cur = cube_run(n, dt, 400)
        if prev is not None:
            for comp in COMPS:
                errs[comp].append(l1(restrict(cur[comp], comp), prev[comp]))
        del prev
        prev = {k: v for k, v in cur.items()}
        del cur
    for comp in COMPS:
        e1, e2 = errs[comp]
        rate = np.log2(e1 / e2)
        a, b, r = ref[("table6", comp)]
        print(f"Table 6 {comp}: {e1:.3e} {e2:.3e} rate {rate:.3f}  (paper {a:.3e} {b:.3e} {r:.2f})", flush=True)
    for comp in COMPS:
        e1, e2 = errs[comp]
        a, b, r = ref[("table6", comp)]
        assert abs(np.log2(e1 / e2) - r) < 0.10, comp
        assert abs(e1 / a - 1) < 0.15 and abs(e2 / b - 1) < 0.15, comp


# Tables 2-4: plane pulses through a homogeneous superconductor or a strip, on the paper's 3-D grids (the
# fields are uniform in x and y, so the L1 means equal those of the 1-D reductions the oracle pins run)
def space_errors(runs):
    """(e_coarse^medium, e_medium^fine) of Ex and By from runs on 128^3, 256^3, 512^3 (finer restricted)."""
    errs = {"Ex": [], "By": []}
    prev = None
    for cur in runs:
        if prev is not None:
            for comp in errs:
                errs[comp].append(l1(restrict(cur[comp], comp), prev[comp]))
        prev = {k: cur[k] for k in errs}
        del cur
    return errs


def check_table(name, errs, tol_err, tol_rate):
    ref = tables()
    for comp, fld in (("Ex", "E"), ("By", "B")):
        e1, e2 = errs[comp]
        a, b, r = ref[(name, fld)]
        rate = np.log2(e1 / e2)
        print(f"{name} {fld}: {e1:.3e} {e2:.3e} rate {rate:.3f}  (paper {a:.3e} {b:.3e} {r:.2f})", flush=True)
        assert abs(e1 / a - 1) < tol_err and abs(e2 / b - 1) < tol_err, (name, fld)
        assert abs(rate - r) < tol_rate, (name, fld)


def test_table2_homogeneous_space_time_convergence():
    runs = (cube_run(n, 0.9 * (1280e-9 / n) / (C0 * np.sqrt(3)), st, region="all", zp=0.0)
            for n, st in ((128, 50), (256, 100), (512, 200)))
    check_table("table2", space_errors(runs), 0.01, 0.02)


def test_table3_strip_time_convergence():
    dt09 = 0.9 * 5e-9 / (C0 * np.sqrt(3))
    sols = [cube_run(256, dt09 * f, st, region="strip") for f, st in ((1.0, 200), (0.5, 400), (0.25, 800))]
    errs = {comp: [l1(sols[1][comp], sols[0][comp]), l1(sols[2][comp], sols[1][comp])] for comp in ("Ex", "By")}
    check_table("table3", errs, 0.10, 0.02)


def test_table4_strip_space_convergence():
    dt = 0.9 * 2.5e-9 / (C0 * np.sqrt(3))
    runs = (cube_run(n, dt, 400, region="strip") for n in (128, 256, 512))
    check_table("table4", space_errors(runs), 0.02, 0.03)


def test_smooth_lambda_keeps_second_order():
    """Sec. 4.3.2: with lambda_L varying smoothly (no sharp interface) the scheme stays second order in
    space, where the strip of Table 4 falls to first order."""
    dt = 0.9 * 2.5e-9 / (C0 * np.sqrt(3))
    errs = space_errors(cube_run(n, dt, 400, region="smooth") for n in (128, 256, 512))
    for comp in ("Ex", "By"):
        e1, e2 = errs[comp]
        print(f"smooth lambda {comp}: {e1:.3e} {e2:.3e} rate {np.log2(e1 / e2):.3f}", flush=True)
        assert np.log2(e1 / e2) > 1.8, comp
