"""The two-step sweep (two time steps per sweep on grids with edge classes) gives the fields and
currents of the fused sweep bit for bit: footprints that do not tile the grid (ragged x, y and z
ranges, grids narrower than a footprint), odd remainders after the four-step groups, CPML slabs and
PEC walls on any axes, both storage types; and it matches the FP64 oracle."""
import numpy as np
import pytest

from paper_2305_13419_amd import workloads
from tests.helpers import compare, run_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def run(wl, steps, dtype, sweep, chunks=None):
    from paper_2305_13419_amd import Simulation
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"])
    sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
    assert sim.edge_classes > 0
    E, H, J = wl["fields"]
    sim.set_fields([np.asarray(a, dtype=npdt) for a in E], [np.asarray(a, dtype=npdt) for a in H],
                   None if J is None else [np.asarray(a, dtype=npdt) for a in J])
    sim.set_sweep(sweep)
    for src in wl.get("sources", []):
        sim.add_source(**src)
    counts = np.zeros(3, dtype=np.int64)
    for c in (chunks or [steps]):
        sim.step(c)
        counts += np.array(sim.sweep_counts())
    torch.cuda.synchronize()
    out = ([t.clone() for t in sim.E + sim.H + sim.J], counts, sim)
    return out


SHAPES = [(256, 64, 32), (200, 50, 40), (130, 33, 17), (62, 10, 9), (40, 7, 70), (300, 12, 5)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", SHAPES)
def test_two_step_equals_fused(shape, dtype):
    wl = workloads.roofline_grid(shape)
    print(f"case: two-step vs fused, {shape}, {dtype}, 11 steps (chunks 8, 3) and 4", flush=True)
    for chunks in ([8, 3], [4]):
        steps = sum(chunks)
        a, ca, sa = run(wl, steps, dtype, "two_step", chunks)
        b, cb, sb = run(wl, steps, dtype, "fused", chunks)
        expect_two = sum(c - c % 4 for c in chunks)
        assert ca[2] == expect_two and cb[2] == 0, (ca, cb)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        sa.close()
        sb.close()


def test_two_step_is_automatic_on_large_periodic_grids():
    """The default policy takes the two-step sweep on a periodic grid with classes past the infinity
    cache (here 3.3 M cells), in both precisions, the fused sweep on a smaller one, still with soft
    sources and probes (which ride along with both steps), and not where the probes' copies of two
    steps do not fit the scratch copy space; on CPML grids in FP64, and in FP32 where the fused sweep's
    rows leave many lanes idle."""
    from paper_2305_13419_amd import Simulation
    small = workloads.roofline_grid((128, 128, 128))
    for dtype in (torch.float32, torch.float64):
        sim = Simulation(small["shape"], small["spacing"], small["dt"], small["theta"], dtype)
        sim.set_materials(*small["maps"])
        sim.set_fields(*small["fields"][:2])
        sim.step(10)
        assert sim.sweep_counts() == (0, 10, 0)
        sim.close()
    wl = workloads.roofline_grid((160, 160, 128))
    E, H, _ = wl["fields"]
    for dtype, expect in ((torch.float32, (0, 2, 8)), (torch.float64, (0, 2, 8))):
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype)
        sim.set_materials(*wl["maps"])
        sim.set_fields(E, H)
        sim.step(10)
        assert sim.sweep_counts() == expect
        sim.add_source(comp=1, box=(0, 160, 0, 160, 9, 10), amplitude=1.0, waveform="sin", freq=2e14)
        sim.step(10)
        assert sim.sweep_counts() == expect
        sim.add_probe(0, (5, 6, 0, 128, 7, 8), 0)
        sim.step(10)
        assert sim.sweep_counts() == expect
        sim.add_probe(1, (0, 160, 0, 160, 7, 10), 0)  # 76 800 values: two copies exceed a half
        sim.step(10)
        assert sim.sweep_counts() == (0, 10, 0)
        sim.close()
    # CPML grids: the two-step sweep in FP64; in FP32 only where 64-cell rows leave a fifth of their
    # lanes idle (nx = 146: 46 of 192; nx = 160: 32 of 192)
    narrow = workloads.roofline_grid((146, 160, 160))
    for w, dtype, expect in ((wl, torch.float32, (0, 10, 0)), (wl, torch.float64, (0, 2, 8)),
                             (narrow, torch.float32, (0, 2, 8))):
        sim = Simulation(w["shape"], w["spacing"], w["dt"], w["theta"], dtype, (None, (4, 4), (8, 8)))
        sim.set_materials(*w["maps"])
        sim.set_fields(*w["fields"][:2])
        sim.step(10)
        assert sim.sweep_counts() == expect, (w["shape"], dtype, sim.sweep_counts())
        sim.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_two_step_matches_oracle(dtype, tol):
    wl = workloads.random_medium((130, 33, 20), seed=19)
    # few distinct materials, so that edge classes bind: the random boxes of the roofline workload; the
    # medium's initial Js (on its own superconducting cells) is dropped with its maps
    wl["maps"] = workloads.roofline_grid((130, 33, 20))["maps"]
    wl["fields"] = (wl["fields"][0], wl["fields"][1], None)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    wl["fields"] = tuple(None if g is None else [np.asarray(a, dtype=npdt).astype(np.float64) for a in g]
                         for g in wl["fields"])
    wl["maps"] = tuple(np.asarray(m, dtype=npdt).astype(np.float64) for m in wl["maps"])
    steps = 12
    a, counts, sim = run(wl, steps, dtype, "two_step")
    assert counts[2] == 12
    Eg, Hg, Jg = sim.integer_time_fields()
    torch.cuda.synchronize()
    g = ([t.double().cpu().numpy() for t in Eg], [t.double().cpu().numpy() for t in Hg],
         [t.double().cpu().numpy() for t in Jg], [])
    sim.close()
    o = run_oracle(wl, steps)
    r = compare(g, o)
    print(f"two-step {dtype} vs oracle, 12 steps: {r}", flush=True)
    assert max(r.values()) <= tol


SOURCES = [
    # a plane source across every footprint row and column, boxes on the x = 0 and y = 0 edges (the
    # wrapped halo columns and rows of neighbouring footprints), two boxes overlapping on Ey
    dict(comp=1, box=(0, 130, 0, 33, 7, 8), amplitude=1.5, waveform="sin", freq=2e14),
    dict(comp=1, box=(60, 64, 10, 20, 3, 15), amplitude=-0.7, waveform="mod_gauss", freq=3e14, t0=2e-15, tw=8e-16),
    dict(comp=0, box=(0, 2, 0, 3, 0, 20), amplitude=0.9, waveform="gauss", t0=1e-15, tw=5e-16),
    dict(comp=2, box=(125, 130, 30, 33, 18, 20), amplitude=2.0, waveform="sin", freq=1e14),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_two_step_with_sources(dtype):
    """Soft sources ride along with both steps of the two-step sweep: the same bits as the fused sweep
    (which adds them to E^{n+1} inside the sweep), and the oracle's fields."""
    wl = workloads.random_medium((130, 33, 20), seed=19)
    wl["maps"] = workloads.roofline_grid((130, 33, 20))["maps"]
    wl["fields"] = (wl["fields"][0], wl["fields"][1], None)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    wl["fields"] = tuple(None if g is None else [np.asarray(a, dtype=npdt).astype(np.float64) for a in g]
                         for g in wl["fields"])
    wl["maps"] = tuple(np.asarray(m, dtype=npdt).astype(np.float64) for m in wl["maps"])
    wl["sources"] = SOURCES
    print(f"case: two-step with sources, (130, 33, 20), {dtype}, 11 steps (chunks 8, 3)", flush=True)
    a, ca, sa = run(wl, 11, dtype, "two_step", [8, 3])
    b, cb, sb = run(wl, 11, dtype, "fused", [8, 3])
    assert ca[2] == 8 and cb[2] == 0, (ca, cb)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    Eg, Hg, Jg = sa.integer_time_fields()
    torch.cuda.synchronize()
    g = ([t.double().cpu().numpy() for t in Eg], [t.double().cpu().numpy() for t in Hg],
         [t.double().cpu().numpy() for t in Jg], [])
    sa.close()
    sb.close()
    o = run_oracle(wl, 11)
    r = compare(g, o)
    print(f"two-step with sources {dtype} vs oracle, 11 steps: {r}", flush=True)
    assert max(r.values()) <= (1e-12 if dtype == torch.float64 else 1e-5)


CPML_CASES = [
    ((130, 33, 40), ((5, 4), None, (3, 6))),
    ((200, 50, 40), (None, (4, 4), None)),
    ((62, 10, 20), ((3, 3), (2, 2), (4, 4))),
    ((256, 64, 32), ((8, 8), None, (8, 8))),
    ((70, 40, 24), ((2, 7), (6, 1), None)),
]


def cpml_workload(shape, pml, seed=29):
    wl = workloads.random_medium(shape, seed=seed, pml=pml)
    wl["maps"] = workloads.roofline_grid(shape)["maps"]  # few distinct materials: edge classes bind
    wl["fields"] = (wl["fields"][0], wl["fields"][1], None)
    return wl


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape,pml", CPML_CASES)
def test_two_step_cpml_equals_fused(shape, pml, dtype):
    """CPML slabs (x-slab columns inside and across footprints, y-slab rows, z-slab planes, slabs on
    every axis of a grid narrower than a footprint) and the PEC walls at their node planes: the
    two-step sweep carries the first step's auxiliary variables in registers and writes the second
    step's to the other set, with the fused sweep's arithmetic."""
    wl = cpml_workload(shape, pml)
    print(f"case: two-step vs fused with CPML, {shape}, pml={pml}, {dtype}, chunks 8, 3", flush=True)
    a, ca, sa = run(wl, 11, dtype, "two_step", [8, 3])
    b, cb, sb = run(wl, 11, dtype, "fused", [8, 3])
    assert ca[2] == 8 and cb[2] == 0, (ca, cb)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    sa.close()
    sb.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_two_step_cpml_matches_oracle(dtype, tol):
    wl = cpml_workload((130, 33, 40), ((5, 4), (3, 3), (3, 6)), seed=37)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    wl["fields"] = tuple(None if g is None else [np.asarray(a, dtype=npdt).astype(np.float64) for a in g]
                         for g in wl["fields"])
    wl["maps"] = tuple(np.asarray(m, dtype=npdt).astype(np.float64) for m in wl["maps"])
    wl["sources"] = [dict(comp=1, box=(20, 21, 0, 33, 5, 35), amplitude=1.0, waveform="mod_gauss", freq=3e14,
                          t0=2e-15, tw=8e-16)]
    steps = 16
    print(f"case: two-step with CPML vs oracle, {dtype}, {steps} steps", flush=True)
    a, counts, sim = run(wl, steps, dtype, "two_step")
    assert counts[2] == 16
    Eg, Hg, Jg = sim.integer_time_fields()
    torch.cuda.synchronize()
    g = ([t.double().cpu().numpy() for t in Eg], [t.double().cpu().numpy() for t in Hg],
         [t.double().cpu().numpy() for t in Jg], [])
    sim.close()
    o = run_oracle(wl, steps)
    r = compare(g, o)
    print(f"two-step with CPML {dtype} vs oracle, {steps} steps: {r}", flush=True)
    assert max(r.values()) <= tol


@pytest.mark.parametrize("theta", [0.5, 0.7])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_two_step_theta_below_one(theta, dtype):
    """theta of Algorithm 1 step 3 below 1 (the centred Ohmic term and a weighted one): the two-step
    sweep equals the fused sweep bit for bit on a periodic grid and on one with CPML slabs, and in FP64
    its integer-time fields match the oracle."""
    cases = (dict(workloads.roofline_grid((130, 40, 24))), cpml_workload((130, 33, 40), ((5, 4), None, (3, 6))))
    for wl in cases:
        wl["theta"] = theta
        print(f"case: two-step vs fused, {wl['shape']}, pml={wl['pml']}, theta {theta}, {dtype}, chunks 8, 3",
              flush=True)
        a, ca, sa = run(wl, 11, dtype, "two_step", [8, 3])
        b, cb, sb = run(wl, 11, dtype, "fused", [8, 3])
        assert ca[2] == 8 and cb[2] == 0, (ca, cb)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        if dtype == torch.float64:
            Eg, Hg, Jg = sa.integer_time_fields()
            torch.cuda.synchronize()
            g = ([t.cpu().numpy() for t in Eg], [t.cpu().numpy() for t in Hg], [t.cpu().numpy() for t in Jg], [])
            o = run_oracle(wl, 11)
            r = compare(g, o)
            print(f"  two-step theta {theta} vs oracle, 11 steps: {r}", flush=True)
            assert max(r.values()) <= 1e-12
        sa.close()
        sb.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(1, 1, 40), (40, 1, 1), (1, 30, 1), (70, 1, 33), (64, 17, 1), (1, 9, 21)])
def test_two_step_degenerate_axes(shape, dtype):
    """Axes of one cell (the wrapped neighbour is the cell itself, so the derivatives along them vanish):
    the two-step sweep, taken on request, equals the fused sweep bit for bit."""
    wl = workloads.roofline_grid(shape)
    print(f"case: two-step vs fused, degenerate {shape}, {dtype}, chunks 8, 3", flush=True)
    a, ca, sa = run(wl, 11, dtype, "two_step", [8, 3])
    b, cb, sb = run(wl, 11, dtype, "fused", [8, 3])
    assert ca[2] == 8 and cb[2] == 0, (ca, cb)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    sa.close()
    sb.close()
