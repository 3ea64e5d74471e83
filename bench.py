"""Throughput of the two-fluid FDTD step on one MI355X.

Workload: the 256^3 roofline grid (dx = 20 nm, periodic, random
superconducting boxes on ~30 % of the cells, E and H ~ N(0, 1)), stepped in
FP64 and in FP32.  A step is one full time step of Algorithm 1.  The product
path is the library's automatic sweep choice (on this grid two time steps per
sweep with edge classes); for comparison the one-step fused sweep (with edge
classes and on the per-cell maps) and the two passes (H pass, E + Js pass).
Also timed: the CPW-shaped 512 x 256 x 128 grid (CPML, two sources, two
probes every step), the adjoint gradient on the half-size CPW workload
(256 x 128 x 64 cells, 4096 steps, 64-step checkpoint segments) against its
checkpointed forward run, and the oracle on a bounded sample on the host
cores.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--n 256] [--no-cpu] [--no-adjoint]
    python bench.py --large      # the 1024 x 512 x 256 workload: FP32 forward 8192 steps and the
                                 # three-level adjoint, plus a finite-difference check of the FP64
                                 # gradient over 512 steps (several minutes)
    python bench.py --table1     # the paper's skin-depth sweep, 12 rows (about 8 minutes)
    python bench.py --paper-cpw  # step rate on the paper's CPW resonator at its own size, 4 film cases
    python bench.py --paper-cpw-q 1,2   # Q and f of film cases 1 and 2 at dz = 200 nm (~6 min per case)
    python bench.py --paper-cpw-q 1 --q-dz 100 --q-end 112   # dz = 100 nm to 112 ps (~15 min)
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s & %HBM roofline, FP64 vs FP32; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0


def sc_edge_fraction(ell):
    """Fraction of edges that carry Js: an edge is superconducting when any of the four cells
    sharing it is (bench-side accounting of the algorithmic bytes)."""
    import numpy as np
    sc = ell > 0
    fr = []
    # Ex edge (i,j,k): cells offset by 0/-1 in y (axis 1 of the array is y) and z (axis 0)
    for axes in ((0, 1), (0, 2), (1, 2)):
        m = sc.copy()
        m |= np.roll(sc, 1, axis=axes[0])
        m |= np.roll(sc, 1, axis=axes[1])
        m |= np.roll(np.roll(sc, 1, axis=axes[0]), 1, axis=axes[1])
        fr.append(m.mean())
    return float(np.mean(fr))


def run_gpu(wl, dtype, steps, warmup, fused=True, classes=True, sweep="auto"):
    import numpy as np
    import torch

    from paper_2305_13419_amd import Simulation

    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"], fused=fused,
                     edge_classes=classes)
    maps = [np.asarray(m, dtype=npdt) for m in wl["maps"]]
    torch.cuda.synchronize()
    tb = time.perf_counter()
    sim.set_materials(*maps)
    torch.cuda.synchronize()
    bind_s = time.perf_counter() - tb
    ncls = sim.edge_classes
    if classes and not ncls:
        raise RuntimeError("edge classes requested but the grid has too many distinct materials")
    E, H, _ = wl["fields"]
    sim.set_fields([np.asarray(a, dtype=npdt) for a in E], [np.asarray(a, dtype=npdt) for a in H])
    sim.set_sweep(sweep)
    sim.step(warmup)
    torch.cuda.synchronize()
    # timed region: K steps, HIP events around every kernel on the launch stream (fused sweep: the
    # first interval is the fused kernel, the second only the gap to the next step)
    t0 = time.perf_counter()
    h_ms, e_ms = sim.profile_step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts = sim.sweep_counts()
    W, bad = sim.energy()
    sim.close()
    return dict(h_ms=h_ms / steps, e_ms=e_ms / steps, step_ms=(h_ms + e_ms) / steps, wall_s=wall,
                nonfinite=int(bad), energy=W, edge_classes=ncls, bind_materials_s=bind_s,
                sweep_counts=dict(zip(("two_pass", "fused", "two_step"), counts)))


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Bandwidth of the runtime's device-to-device copy (torch copy_ of `nbytes`, read + write bytes per
    second, GB/s), timed with events around `reps` copies: a reference rate on this GPU."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


KERNEL_SOURCES = ("kernels_fwd.hip", "fdtd_common.h", "tfl_internal.h")


def kernel_code_hash():
    """Hash of the forward kernels' code: their source and the headers they include, with comments,
    indentation and blank lines removed (a change of comments leaves the kernels as measured)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2305_13419_amd", "csrc", name)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(ln.strip() for ln in text.splitlines() if ln.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(dtype_name, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None when the
    kernels' code changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "forward_kernels_roofline_256cube.md")
    if not os.path.exists(path):
        return None
    code = kernel_code_hash()
    for line in open(path):
        m = re.match(r"TRAFFIC (\w+) (\w+) bytes_per_launch=(\S+) kernel_code=(\w+)", line.strip())
        if m and m.group(1) == dtype_name and m.group(2) == kernel:
            return float(m.group(3)) if m.group(4) == code else None
    return None


def adjoint_ratio(dtype, seg=64):
    """Wall time of the reverse sweep over that of the checkpointed forward run (half-size CPW)."""
    import numpy as np
    import torch

    from paper_2305_13419_amd import Simulation, workloads

    wl = workloads.cpw_grid(2)
    N = wl["steps"]
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"])
    sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
    z = [np.zeros(sim.shape3, dtype=npdt)] * 3
    for s in wl["sources"]:
        sim.add_source(**s)
    obj = wl["objective"]
    ckpt, snap, work = sim.adjoint_buffers(N, seg)
    best = None
    for _ in range(2):  # the first pass warms up allocations and code objects
        sim.set_fields(z, z, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = sim.forward_checkpointed(obj, N, seg, ckpt)
        t1 = time.perf_counter()
        sim.adjoint(obj, N, seg, ckpt, F, snap, work)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        best = (t1 - t0, t2 - t1)
    sim.close()
    return dict(forward_s=best[0], adjoint_s=best[1], ratio=best[1] / best[0], steps=N, seg=seg,
                workload=wl["name"])


def large_run(steps=8192, seg=512, seg2=32, fd_steps=512, fd_cells=4):
    """FP32 forward + three-level adjoint on the large grid, then central differences of the FP64
    forward (three-level adjoint over fd_steps) at fd_cells cells per map."""
    import numpy as np
    import torch

    from paper_2305_13419_amd import Simulation, workloads

    wl = workloads.large_mixed_grid(steps=steps)
    n = int(np.prod(wl["shape"]))
    # the objective's frequency, frozen once: the peak of |DFT| of the objective line over an unperturbed
    # FP64 run of the same length (as for the half-size CPW)
    print("# large: FP64 run for the objective frequency", file=sys.stderr, flush=True)
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], torch.float64, wl["pml"])
    sim.set_materials(*wl["maps"])
    for s in wl["sources"]:
        sim.add_source(**s)
    z = [torch.zeros(sim.shape3, dtype=torch.float64, device="cuda")] * 3
    sim.set_fields(z, z, z)
    pid = sim.add_probe(wl["objective"][0], wl["objective"][1], steps + 1)
    sim.step(steps)
    series = np.asarray(sim.probe(pid)[0])
    sim.close()
    del sim, z
    torch.cuda.empty_cache()
    freqs = np.linspace(0.25 * wl["freq"], 2.0 * wl["freq"], 3501)
    t = np.arange(series.size) * wl["dt"]
    f0 = float(freqs[np.argmax(np.abs(np.exp(-2j * np.pi * np.outer(freqs, t)) @ series))])
    obj = (wl["objective"][0], wl["objective"][1], f0)
    out = {"workload": wl["name"], "steps": steps, "seg": seg, "seg2": seg2, "objective_f0": f0,
           "source_f": wl["freq"]}

    def make(dtype, npdt):
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"])
        sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
        for s in wl["sources"]:
            sim.add_source(**s)
        z = [torch.zeros(sim.shape3, dtype=dtype, device="cuda")] * 3
        sim.set_fields(z, z, z)
        return sim

    print("# large: FP32 forward and three-level adjoint", file=sys.stderr, flush=True)
    torch.cuda.reset_peak_memory_stats()
    sim = make(torch.float32, np.float32)
    ckpt, ckpt2, snap, work = sim.adjoint_nested_buffers(steps, seg, seg2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = sim.forward_checkpointed(obj, steps, seg, ckpt)
    t1 = time.perf_counter()
    print(f"# large FP32: forward {t1 - t0:.1f} s; adjoint", file=sys.stderr, flush=True)
    gl, gs = sim.adjoint_nested(obj, steps, seg, seg2, ckpt, F, ckpt2, snap, work)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["f32"] = dict(forward_s=t1 - t0, forward_Gcells=n * steps / (t1 - t0) / 1e9, adjoint_s=t2 - t1,
                      ratio=(t2 - t1) / (t1 - t0), J=abs(F) ** 2,
                      peak_GB=torch.cuda.max_memory_allocated() / 1e9,
                      grad_finite=bool(torch.isfinite(gl).all() and torch.isfinite(gs).all()))
    print(f"# large FP32: {out['f32']}", file=sys.stderr, flush=True)
    sim.close()
    del sim, ckpt, ckpt2, snap, work, gl, gs
    torch.cuda.empty_cache()

    print(f"# large: FP64 gradient over {fd_steps} steps and central differences", file=sys.stderr, flush=True)
    sim = make(torch.float64, np.float64)
    s1, s2 = 128, 16
    ckpt, ckpt2, snap, work = sim.adjoint_nested_buffers(fd_steps, s1, s2)
    F = sim.forward_checkpointed(obj, fd_steps, s1, ckpt)
    gl, gs = sim.adjoint_nested(obj, fd_steps, s1, s2, ckpt, F, ckpt2, snap, work)
    gl, gs = gl.cpu().numpy(), gs.cpu().numpy()
    del ckpt, ckpt2, snap, work
    torch.cuda.empty_cache()
    J0 = abs(F) ** 2
    fpid = sim.add_probe(obj[0], obj[1], 0, [obj[2]])
    eps, sig, ell = wl["maps"]
    dev = [torch.tensor(m, device="cuda") for m in (eps, sig, ell)]

    def J_of(mi, cell, delta):
        d = dev[mi].clone()
        d[cell] += delta
        maps = [dev[0], d if mi == 1 else dev[1], d if mi == 2 else dev[2]]
        sim.set_materials(*maps)
        z = [torch.zeros(sim.shape3, dtype=torch.float64, device="cuda")] * 3
        sim.set_fields(z, z, z)
        sim._probes[fpid][1].zero_()
        sim.step(fd_steps)
        return abs(sim.probe(fpid)[1][0]) ** 2

    rng = np.random.default_rng(5)
    errs = {}
    hrel = 1e-4
    for name, g, m, ref, mi in (("ell", gl, ell, 1e14, 2), ("sigma", gs, sig, 1e4, 1)):
        dJ = np.abs(g) * hrel * np.maximum(np.abs(m), ref) / J0
        ok = (m > 0) & (dJ >= 1e-2 * dJ[m > 0].max())
        cells = np.argwhere(ok)
        e = []
        for c in cells[rng.choice(len(cells), fd_cells, replace=False)]:
            c = tuple(int(v) for v in c)
            h = hrel * max(abs(m[c]), ref)
            fd = (J_of(mi, c, h) - J_of(mi, c, -h)) / (2 * h)
            e.append(abs(g[c] - fd) / abs(fd))
        errs[name] = max(e)
    out["fd_fp64"] = dict(steps=fd_steps, seg=s1, seg2=s2, cells_per_map=fd_cells, max_rel_err=errs)
    sim.close()
    return out


def cpu_baseline(wl, steps):
    """The FP64 CPU oracle on the same grid, a bounded number of steps."""
    import numpy as np

    from oracle.oracle import OracleSim

    E, H, _ = wl["fields"]
    o = OracleSim(wl["shape"], wl["spacing"], wl["dt"], wl["theta"])
    o.set_materials(*wl["maps"])
    o.set_fields(E, [h * 1.25663706212e-6 for h in H], [np.zeros_like(E[0])] * 3)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    n = wl["shape"][0] * wl["shape"][1] * wl["shape"][2]
    from oracle import oracle as oracle_mod
    cores = oracle_mod.threads()  # the OpenMP threads the oracle's grid sweeps run on
    return dict(value=n * steps / dt / 1e9, unit="Gcell-updates/s", cores=cores, kind="oracle",
                sample=f"{steps} FP64 steps of the same {wl['shape'][0]}^3 grid ({dt:.1f} s)")


def cpw_rate(steps=200, warmup=20):
    """Step rate on the CPW-resonator-shaped grid (512 x 256 x 128, CPML on x and z, soft sources and two
    FP64 probes every step): FP32 fields (the workload's precision) and FP64, with the kernels' own
    HIP-event times (the sources and probes ride along with the sweeps; on the two passes the first
    launch is the H pass and the rest the E pass), the steps per sweep path and the wall time."""
    import numpy as np
    import torch

    from paper_2305_13419_amd import Simulation, workloads

    wl = workloads.cpw_grid(1)
    n = int(np.prod(wl["shape"]))
    out = {"workload": wl["name"] + " (CPML x, z; 2 soft sources, 2 FP64 probes)", "cells": n, "steps": steps}
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        npdt = np.float64 if dt == torch.float64 else np.float32
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dt, wl["pml"])
        sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
        z = [np.zeros(sim.shape3, dtype=npdt)] * 3
        sim.set_fields(z, z, z)
        for s in wl["sources"]:
            sim.add_source(**s)
        for p in wl["probes"]:
            sim.add_probe(p["comp"], p["box"], steps + warmup + 1)
        sim.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h_ms, e_ms = sim.profile_step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = (h_ms + e_ms) / steps
        paths = dict(zip(("two_pass", "fused", "two_step"), sim.sweep_counts()))
        sim.close()
        out[name] = dict(value=n / (ms * 1e-3) / 1e9, unit="Gcell-updates/s", ms_per_step=ms,
                         first_launch_ms=h_ms / steps, rest_ms=e_ms / steps, paths=paths,
                         wall_ms_per_step=wall / steps * 1e3)
    return out


def table1_run():
    """The paper's skin-depth sweep (Sec. 4.1, Table 1): all twelve (sigma, f) rows in FP64 on 1-D lines
    with CPML ends, five periods each (the undamped 100 THz row, 16 % below the cutoff, also after 200
    periods); skin depth from the steady-state amplitudes at the source and at z0."""
    import numpy as np
    import torch

    from oracle import closed_forms as cf
    from paper_2305_13419_amd import Simulation, workloads

    ell = 1.0 / (400e-9) ** 2
    rows = []
    runs = [(s, f, p, 5) for s, f, p in workloads.TABLE1_ROWS] + [(0.0, 1e14, 739, 200)]
    for sigma, freq, paper, periods in runs:
        theory = float(cf.skin_depth(freq, 1.0, sigma, ell))
        wl = workloads.table1_grid(sigma, freq, theory, periods=periods)
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], 1.0, torch.float64, wl["pml"])
        sim.set_materials(*wl["maps"])
        for src in wl["sources"]:
            sim.add_source(**src)
        pids = [sim.add_probe(p["comp"], p["box"], wl["steps"] + 1) for p in wl["probes"]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        left = wl["steps"]
        while left > 0:
            c = min(left, 1000000)
            sim.step(c)
            left -= c
            torch.cuda.synchronize()
            print(f"# table1 sigma={sigma:g} f={freq:g}: {wl['steps'] - left} / {wl['steps']} steps, "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
        el = time.perf_counter() - t0
        fit = 50 if periods > 5 else 2
        a0, a1 = (workloads.steady_amplitude(sim.probe(p)[0], wl["dt"], freq, periods=fit) for p in pids)
        sim.close()
        rows.append(dict(sigma=sigma, f=freq, periods=periods, steps=wl["steps"], seconds=el,
                         computed_nm=wl["z0"] / np.log(a0 / a1) * 1e9,
                         discrete_nm=float(cf.discrete_skin_depth(freq, 10e-9, wl["dt"], 1.0, 1.0, sigma, ell)) * 1e9,
                         theory_nm=theory * 1e9, paper_computed_nm=paper))
        print(f"# {rows[-1]}", file=sys.stderr, flush=True)
    return rows


def paper_cpw_run(steps=200, warmup=10, cases=(1, 2, 3, 4), fused=True):
    """Step rate on the paper's CPW resonator at its own size (196 M cells with the CPML slabs), each
    film case, FP32 and FP64, against the paper's ~0.05 s per step on 32 A100 GPUs (fused=False: the
    two passes instead of the fused sweep)."""
    import numpy as np
    import torch

    from paper_2305_13419_amd import Simulation, workloads

    rows = []
    for case in cases:
        wl = workloads.paper_cpw_grid(case)
        for dtype, npdt in ((torch.float32, np.float32), (torch.float64, np.float64)):
            sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"], fused=fused)
            sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
            for src in wl["sources"]:
                sim.add_source(**src)
            pids = [sim.add_probe(p["comp"], p["box"], steps + warmup + 1) for p in wl["probes"]]
            sim.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            W, bad = sim.energy()
            series_ok = bool(np.all(np.isfinite(sim.probe(pids[1])[0])))
            sim.close()
            n = int(np.prod(wl["shape"]))
            rows.append(dict(case=case, dtype=str(dtype)[6:], fused=fused, cells=n, steps=steps, ms_per_step=el / steps * 1e3,
                             Gcells=n * steps / el / 1e9, dt_s=wl["dt"], nonfinite=int(bad), probes_finite=series_ok,
                             paper_s_per_step=0.05, speedup_per_step=0.05 / (el / steps)))
            print(f"# {rows[-1]}", file=sys.stderr, flush=True)
            del sim
            torch.cuda.empty_cache()
    return rows


def paper_cpw_q_run(cases=(1, 2, 3, 4), dz=200e-9, t_end=134e-12, t_fit=80e-12, fit_ends=None, save_dir=None,
                    film_sigma=None):
    """Q and resonance of the paper's CPW (Sec. 5, Table 7) at a coarser z resolution (dz = 200 nm: the
    film one cell thick; 100 nm: two cells; the paper's 50 nm needs 850 000 steps of 196 M cells): FP32
    fields, FP64 probe series, run to t_end; ESPRIT (and the linear predictor) on the Ex probe at the
    resonator's front edge over [t_fit, te] for each te of fit_ends (default: t_end), decimated to ~32
    samples per period of the DFT peak."""
    import numpy as np
    import torch

    from paper_2305_13419_amd import Simulation, workloads

    rows = []
    for case in cases:
        wl = workloads.paper_cpw_grid(case, dz=dz, film_sigma=film_sigma)
        steps = int(np.ceil(t_end / wl["dt"]))
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], torch.float32, wl["pml"])
        sim.set_materials(*[np.asarray(m, dtype=np.float32) for m in wl["maps"]])
        for src in wl["sources"]:
            sim.add_source(**src)
        pids = [sim.add_probe(p["comp"], p["box"], steps + 1) for p in wl["probes"]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            c = min(steps - done, 20000)
            sim.step(c)
            done += c
            torch.cuda.synchronize()
            print(f"# paper cpw case {case}: {done} / {steps} steps, {time.perf_counter() - t0:.0f} s", file=sys.stderr,
                  flush=True)
        el = time.perf_counter() - t0
        series = np.asarray(sim.probe(pids[1])[0])
        start = int(t_fit / wl["dt"])
        fits = []
        for te in (fit_ends or (t_end,)):
            stop = min(steps, int(np.ceil(te / wl["dt"])))
            tail = series[start:stop + 1]
            freqs = np.linspace(50e9, 150e9, 2001)
            t = np.arange(tail.size) * wl["dt"]
            spec = np.abs(np.exp(-2j * np.pi * np.outer(freqs, t)) @ tail)
            fh = float(freqs[np.argmax(spec)])
            decim = max(1, int(round(1.0 / fh / wl["dt"] / 32)))
            count = (stop - start) // decim
            esp = sim.esprit_fit(pids[1], start, count, decim, 0, 0, f_hint=fh)
            lp = sim.ringdown_fit(pids[1], start, count, decim, 0, f_hint=fh)
            fits.append(dict(window_ps=[t_fit * 1e12, te * 1e12], dft_peak_GHz=fh / 1e9,
                             esprit=dict(f_GHz=esp["f0"] / 1e9, Q=esp["Q"], order=esp["order"]),
                             linear_prediction=dict(f_GHz=lp["f0"] / 1e9, Q=lp["Q"], order=lp["order"]),
                             window=dict(start=start, count=count, decim=decim)))
        sim.close()
        _, _, q_paper, f_paper = workloads.PAPER_CPW_CASES[case]
        rows.append(dict(case=case, dz=dz, cells=int(np.prod(wl["shape"])), steps=steps, seconds=el, fits=fits,
                         paper=dict(f_GHz=f_paper, Q=q_paper)))
        print(f"# {rows[-1]}", file=sys.stderr, flush=True)
        if save_dir:  # every 16th sample of the FP64 probe series, for fits outside the library
            os.makedirs(save_dir, exist_ok=True)
            np.save(os.path.join(save_dir, f"paper_cpw_q_case{case}_dz{int(round(dz * 1e9))}nm.npy"), series[::16])
        del sim
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--no-cpw", action="store_true", help="skip the CPW-shaped grid's step rate")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--large", action="store_true")
    ap.add_argument("--table1", action="store_true")
    ap.add_argument("--paper-cpw", action="store_true")
    ap.add_argument("--paper-cpw-q", type=str, default="", help="comma-separated film cases, e.g. 1,2")
    ap.add_argument("--q-dz", type=float, default=200.0, help="cell size along z of the Q runs (nm)")
    ap.add_argument("--q-end", type=float, default=134.0, help="end time of the Q runs (ps)")
    ap.add_argument("--q-fit-ends", type=str, default="", help="comma-separated ends of the fit windows (ps)")
    ap.add_argument("--save-series", type=str, default="", help="directory for the Q runs' probe series (.npy)")
    ap.add_argument("--q-film-sigma", type=float, default=None, help="film conductivity of the Q runs (S/m)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2305_13419_amd import workloads

    if args.large:
        print(json.dumps({"metric": METRIC, "large": large_run()}), flush=True)
        return
    if args.paper_cpw_q:
        cases = tuple(int(c) for c in args.paper_cpw_q.split(","))
        ends = tuple(float(e) * 1e-12 for e in args.q_fit_ends.split(",")) if args.q_fit_ends else None
        q = paper_cpw_q_run(cases, dz=args.q_dz * 1e-9, t_end=args.q_end * 1e-12, fit_ends=ends,
                            save_dir=args.save_series, film_sigma=args.q_film_sigma)
        print(json.dumps({"metric": f"Q and f of the paper's CPW at dz = {args.q_dz:g} nm", "paper_cpw_q": q}),
              flush=True)
        return
    if args.paper_cpw:
        print(json.dumps({"metric": "step rate on the paper's CPW resonator", "paper_cpw": paper_cpw_run()}),
              flush=True)
        return
    if args.table1:
        print(json.dumps({"metric": "skin depth (nm), Table 1 sweep", "table1": table1_run()}), flush=True)
        return

    wl = workloads.roofline_grid(args.n, steps=args.steps)
    ncell = args.n**3
    fJ = sc_edge_fraction(wl["maps"][2])
    res = {}
    # product path: the automatic sweep choice, i.e. two time steps per sweep with edge classes on this
    # periodic grid; beside it one step per sweep (the fused sweep) with classes and on the per-cell
    # maps, and the two passes (H pass, E pass) with classes
    modes = {"auto": (True, True, "auto"), "fused": (True, True, "fused"), "fused_maps": (True, False, "fused"),
             "two_pass": (False, True, "two_pass")}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        for mode, (fused, classes, sweep) in modes.items():
            print(f"# {name} {mode}: {args.warmup} warm-up + {args.steps} timed steps on {wl['name']}",
                  file=sys.stderr, flush=True)
            res[name, mode] = run_gpu(wl, dt, args.steps, args.warmup, fused, classes, sweep)
    copy_gbs = copy_bandwidth()
    out = {}
    for name, w in (("f64", 8), ("f32", 4)):
        # per cell: E, H read and written (fused) or E read and written, H read (E pass); Js read and
        # written on the f_J superconducting edges; the E update's coefficients as three 16-bit edge
        # classes (6 B) or three per-cell maps (3 w)
        f_cell = w * (12 + 6 * fJ) + 6
        m_cell = w * (15 + 6 * fJ)
        e_cell = w * (9 + 6 * fJ) + 6
        h_cell = w * 9                             # H pass: E, H read; H written

        # the method's minimum bytes per cell-update (E and H read and written once, Js read and written
        # on the superconducting edges, three per-cell map words): the per-unit figure `achieved` uses
        method_cell = w * (15 + 6 * fJ)

        def roof(kernel, ms, cell, traffic_key, steps_per_launch=1):
            """achieved = the method's minimum bytes per cell-update x the cell-updates of one launch / the
            launch's average duration; kernel_* = the same with the bytes this kernel itself must move
            (edge classes instead of maps: fewer than the method's minimum).  A launch that is part of a
            step (steps_per_launch=0: the E pass) is measured by its own bytes."""
            per_launch = method_cell * ncell * steps_per_launch if steps_per_launch else cell * ncell
            gbs = per_launch / (ms * 1e-3) / 1e9
            kgbs = cell * ncell / (ms * 1e-3) / 1e9
            traffic = measured_traffic(name, traffic_key)
            return dict(bound="hbm", kernel=kernel, achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=gbs / HBM_PEAK_GBS, traffic=traffic,
                        bytes_per_cell_update=method_cell if steps_per_launch else None,
                        algorithmic_bytes_per_launch=per_launch,
                        kernel_bytes_per_cell=cell, kernel_achieved=kgbs, kernel_frac=kgbs / HBM_PEAK_GBS,
                        # measured HBM bytes per launch over the launch time, and the kernel's own rate
                        # against the runtime's device-to-device copy on this GPU
                        traffic_GBs=None if traffic is None else traffic / (ms * 1e-3) / 1e9,
                        runtime_copy_GBs=copy_gbs, frac_of_runtime_copy=kgbs / copy_gbs)

        a_, r, m, t = res[name, "auto"], res[name, "fused"], res[name, "fused_maps"], res[name, "two_pass"]
        # the two-step sweep: one launch per two steps, reading and writing E, H, Js and the classes once
        two = a_["sweep_counts"]["two_step"] == args.steps
        spl = 2 if two else 1
        out[name] = dict(
            value=ncell / (a_["step_ms"] * 1e-3) / 1e9, ms_per_step=a_["step_ms"], sweep_counts=a_["sweep_counts"],
            nonfinite=a_["nonfinite"], edge_classes=a_["edge_classes"], bind_materials_s=a_["bind_materials_s"],
            roofline=dict(roof("two_step_kernel (edge classes)" if two else "fused_step_kernel (edge classes)",
                               a_["h_ms"] * spl, f_cell, "two_step_kernel" if two else "fused_step_kernel", spl),
                          steps_per_launch=spl, launch_ms=a_["h_ms"] * spl),
            fused=dict(
                value=ncell / (r["step_ms"] * 1e-3) / 1e9, ms_per_step=r["step_ms"], fused_step_ms=r["h_ms"],
                nonfinite=r["nonfinite"], sweep_counts=r["sweep_counts"],
                roofline=roof("fused_step_kernel (edge classes)", r["h_ms"], f_cell, "fused_step_kernel")),
            maps_path=dict(
                value=ncell / (m["step_ms"] * 1e-3) / 1e9, ms_per_step=m["step_ms"], nonfinite=m["nonfinite"],
                roofline=roof("fused_step_kernel (maps)", m["h_ms"], m_cell, "fused_step_kernel_maps")),
            two_pass=dict(
                value=ncell / (t["step_ms"] * 1e-3) / 1e9, ms_per_step=t["step_ms"], h_pass_ms=t["h_ms"],
                e_pass_ms=t["e_ms"], h_pass_GBs=h_cell * ncell / (t["h_ms"] * 1e-3) / 1e9, nonfinite=t["nonfinite"],
                roofline=roof("e_pass_kernel (edge classes)", t["e_ms"], e_cell, "e_pass_kernel", 0)),
        )
    f64 = out["f64"]
    line = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"] + " roofline grid, dx=20nm, periodic, ~30% SC boxes (seed 2), "
                               "E,H~N(0,1), theta=1", "cells": ncell, "sc_edge_fraction": fJ},
        "roofline": f64["roofline"],
        "f64": {k: v for k, v in f64.items() if k != "roofline"},
        "f32": out["f32"],
    }
    if not args.no_cpw:
        print("# cpw-shaped grid step rate", file=sys.stderr, flush=True)
        line["cpw_shaped"] = cpw_rate()
    if not args.no_adjoint:
        ratios = {}
        for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
            print(f"# adjoint/forward ratio, {name}", file=sys.stderr, flush=True)
            ratios[name] = adjoint_ratio(dt)
        line["adjoint_forward_ratio"] = {k: v["ratio"] for k, v in ratios.items()}
        line["adjoint"] = ratios
    if not args.no_cpu:
        print(f"# cpu_baseline: oracle, {args.cpu_steps} steps", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
