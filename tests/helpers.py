"""Run one workload on the HIP path and on the FP64 oracle, and compare."""
import numpy as np

from oracle.oracle import OracleSim

MU0 = 1.25663706212e-6
WAVE_KIND = {"sin": 0, "gauss": 1, "mod_gauss": 2}


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def fields_of(wl, dtype=np.float64):
    """Initial fields (E, H, J) cast through `dtype` (the FP32 path starts from FP32-rounded data)."""
    nz, ny, nx = wl["shape"][2], wl["shape"][1], wl["shape"][0]
    z = [np.zeros((nz, ny, nx)) for _ in range(3)]
    F = wl.get("fields")
    if F is None:
        F = (z, z, None)
    E, H, J = F
    J = J if J is not None else z
    cast = lambda a: np.asarray(a, dtype=dtype).astype(np.float64)  # noqa: E731
    return [cast(a) for a in E], [cast(a) for a in H], [cast(a) for a in J]


def maps_of(wl, dtype=np.float64):
    return [np.asarray(m, dtype=dtype).astype(np.float64) for m in wl["maps"]]


def run_oracle(wl, steps, dtype=np.float64, probe_cap=None, chunk=None):
    """Oracle run from the inputs rounded to `dtype`.  Returns (E, H, J, probes).  With `chunk`, the
    steps run in chunks of that many with a progress line after each (long runs)."""
    pml = wl["pml"]
    o = OracleSim(wl["shape"], wl["spacing"], wl["dt"], wl["theta"],
                  pml=[0 if p is None else 1 for p in pml], npml=[(0, 0) if p is None else p for p in pml],
                  **wl.get("pml_params", {}))
    o.set_materials(*maps_of(wl, dtype))
    E, H, J = fields_of(wl, dtype)
    o.set_fields(E, [h * MU0 for h in H], J)
    for s in wl["sources"]:
        o.add_source(s["comp"], s["box"], s["amplitude"], WAVE_KIND[s.get("waveform", "sin")], s.get("freq", 0.0),
                     s.get("t0", 0.0), s.get("tw", 1.0))
    pids = [o.add_probe(p["comp"], p["box"], probe_cap or steps + 1, p.get("freqs", ())) for p in wl["probes"]]
    if chunk:
        import time
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            n = min(chunk, steps - done)
            o.step(n)
            done += n
            print(f"    oracle {done}/{steps} steps, {time.perf_counter() - t0:.0f} s", flush=True)
    else:
        o.step(steps)
    Eo, Bo, Jo = o.get_fields()
    return Eo, [b / MU0 for b in Bo], Jo, [o.probe(p) for p in pids]


def run_gpu(wl, steps, dtype, probe_cap=None, chunks=None):
    """HIP-path run through the C ABI.  Returns (E, H, J, probes) at integer time as float64 numpy."""
    import torch

    from paper_2305_13419_amd import Simulation

    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"],
                     **wl.get("pml_params", {}))
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
    E, H, J = fields_of(wl, npdt)
    sim.set_fields(E, H, J)
    for s in wl["sources"]:
        sim.add_source(**s)
    pids = [sim.add_probe(p["comp"], p["box"], probe_cap or steps + 1, p.get("freqs", ())) for p in wl["probes"]]
    if chunks:
        done = 0
        for c in chunks:
            sim.step(c)
            done += c
        assert done == steps
    else:
        sim.step(steps)
    Eg, Hg, Jg = sim.integer_time_fields()
    torch.cuda.synchronize()
    out = ([t.double().cpu().numpy() for t in Eg], [t.double().cpu().numpy() for t in Hg],
           [t.double().cpu().numpy() for t in Jg], [sim.probe(p) for p in pids])
    sim.close()
    return out


def compare(g, o):
    """Relative L2 per field group (E, H, J) and per probe (series, dft)."""
    res = {}
    for name, a, b in (("E", g[0], o[0]), ("H", g[1], o[1]), ("J", g[2], o[2])):
        res[name] = rel_l2(np.stack(a), np.stack(b))
    for q, (pg, po) in enumerate(zip(g[3], o[3])):
        res[f"probe{q}"] = rel_l2(pg[0], po[0])
        if len(po[1]):
            res[f"dft{q}"] = rel_l2(pg[1], po[1])
    return res


def max_abs_rel(a, b):
    """max |a - b| over the elements divided by max |b|: an error confined to a few cells (a CPML slab,
    a film) that the relative L2 over a large grid would average away shows here."""
    mb = float(np.max(np.abs(b))) if np.size(b) else 0.0
    d = float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(b) else 0.0
    return d / mb if mb > 0 else d


def compare_full(g, o):
    """compare() plus the element-wise max-abs error (max_abs_rel) of every field group and probe."""
    res = compare(g, o)
    for name, a, b in (("E", g[0], o[0]), ("H", g[1], o[1]), ("J", g[2], o[2])):
        res[f"maxabs_{name}"] = max_abs_rel(np.stack(a), np.stack(b))
    for q, (pg, po) in enumerate(zip(g[3], o[3])):
        res[f"maxabs_probe{q}"] = max_abs_rel(pg[0], po[0])
    return res


def rounded_inputs(wl, dtype=np.float32):
    """The workload with its maps and initial fields rounded to `dtype` (kept as float64 arrays), so that
    an FP64 run, an FP32 run and the oracle all start from the same values and one oracle run serves
    both comparisons (rounding to FP32 twice changes nothing)."""
    out = dict(wl)
    out["maps"] = tuple(np.asarray(m, dtype=dtype).astype(np.float64) for m in wl["maps"])
    if wl.get("fields") is not None:
        E, H, J = wl["fields"]
        r = lambda grp: None if grp is None else [np.asarray(a, dtype=dtype).astype(np.float64) for a in grp]  # noqa
        out["fields"] = (r(E), r(H), r(J))
    return out
