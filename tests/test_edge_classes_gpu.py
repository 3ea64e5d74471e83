"""Edge-coefficient classes (tfl_bind_edge_classes): the forward sweeps and the adjoint edge sweep
read one 16-bit class per edge and a table of coefficients instead of the per-cell maps.  The
table is computed by the sweeps' own coefficient code, so fields, currents, probe series and
gradients must equal those of the maps path bit for bit."""
import numpy as np
import pytest

from paper_2305_13419_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def boxes_grid(shape, pml, seed=3, theta=1.0):
    """Random superconducting boxes (few distinct materials, as in the roofline workload) on an
    eps_r = 11.7 substrate in the lower third, random fields."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    er = np.ones((nz, ny, nx))
    er[: nz // 3] = 11.7
    maps = workloads.random_boxes(shape, rng, side=(2, 9), eps_r=er)
    d = (20e-9, 20e-9, 20e-9)
    fields = tuple([rng.standard_normal((nz, ny, nx)) for _ in range(3)] for _ in range(3))
    return dict(shape=shape, spacing=d, dt=workloads.courant_dt(d, 1.0 / (50e-9) ** 2, 0.95), theta=theta,
                pml=pml, maps=maps, fields=fields)


def run(wl, steps, dtype, classes, fused=True, chunks=None):
    from paper_2305_13419_amd import Simulation
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"], fused=fused,
                     edge_classes=classes)
    sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
    ncls = sim.edge_classes
    assert (ncls > 0) == classes
    E, H, J = wl["fields"]
    sim.set_fields(*[[np.asarray(a, dtype=npdt) for a in grp] for grp in (E, H, J)])
    nx, ny, nz = wl["shape"]
    sim.add_source(comp=1, box=(nx // 2, nx // 2 + 1, 0, ny, nz // 4, nz // 2), amplitude=2.0,
                   waveform="mod_gauss", freq=3e14, t0=2e-15, tw=8e-16)
    pid = sim.add_probe(1, (2 * nx // 3, 2 * nx // 3 + 1, 0, ny, 0, nz), steps + 1, [3e14])
    for c in (chunks or [steps]):
        sim.step(c)
    torch.cuda.synchronize()
    out = [t.clone() for t in sim.E + sim.H + sim.J] + [torch.tensor(np.asarray(sim.probe(pid)[0]))]
    sim.close()
    return out, ncls


def assert_same(a, b):
    worst = max(float(((x.double() - y.double()).abs().max() / y.double().abs().max().clamp_min(1e-300)))
                for x, y in zip(a, b))
    print(f"  max relative difference {worst:.3e}", flush=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


GRIDS = {
    "periodic boxes": lambda: boxes_grid((70, 36, 44), (None, None, None)),
    "cpml boxes": lambda: boxes_grid((66, 40, 38), ((6, 5), None, (4, 7)), theta=0.7),
    "random medium": lambda: workloads.random_medium((21, 18, 16), seed=9, pml=((3, 3), (2, 4), None)),
}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("grid", list(GRIDS))
@pytest.mark.parametrize("fused", [True, False])
def test_classes_equal_maps(grid, dtype, fused):
    wl = GRIDS[grid]()
    if wl["fields"] is None or wl["fields"][2] is None:
        rng = np.random.default_rng(4)
        nx, ny, nz = wl["shape"]
        wl["fields"] = tuple([rng.standard_normal((nz, ny, nx)) for _ in range(3)] for _ in range(3))
    print(f"case: classes vs maps, {grid} {wl['shape']}, {dtype}, fused={fused}", flush=True)
    a, ncls = run(wl, 9, dtype, True, fused, chunks=[4, 5])
    b, _ = run(wl, 9, dtype, False, fused, chunks=[4, 5])
    print(f"  {ncls} classes", flush=True)
    assert_same(a, b)


def test_too_many_materials_stays_on_maps():
    """Per-cell random materials on 55 440 cells give more distinct edges than the class table holds:
    the binding reports it and the simulation runs on the maps."""
    from paper_2305_13419_amd import Simulation
    wl = workloads.random_medium((66, 21, 40), seed=5)
    print("case: class table overflow, random medium (66, 21, 40)", flush=True)
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], torch.float64, wl["pml"])
    sim.set_materials(*wl["maps"])
    assert sim.edge_classes == 0 and sim.class_buffer is None
    sim.set_fields(*wl["fields"])
    sim.step(3)
    torch.cuda.synchronize()
    assert all(torch.isfinite(t).all() for t in sim.E)
    sim.close()


def test_rebinding_materials_rebuilds_classes():
    """Classes are a snapshot of the maps: new maps bound later must be the ones the sweeps use."""
    from paper_2305_13419_amd import Simulation
    wl = boxes_grid((64, 20, 24), (None, None, None), seed=8)
    wl2 = boxes_grid((64, 20, 24), (None, None, None), seed=9)
    print("case: rebinding materials, (64, 20, 24)", flush=True)
    outs = []
    for classes in (True, False):
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], torch.float64, wl["pml"],
                         edge_classes=classes)
        sim.set_materials(*wl["maps"])
        sim.set_fields(*wl["fields"])
        sim.step(3)
        sim.set_materials(*wl2["maps"])
        assert (sim.edge_classes > 0) == classes
        sim.step(4)
        torch.cuda.synchronize()
        outs.append([t.clone() for t in sim.E + sim.H + sim.J])
        sim.close()
    assert_same(*outs)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_adjoint_with_classes_equals_maps(dtype):
    from tests.test_adjoint_gpu import gpu_adjoint
    wl = boxes_grid((40, 12, 36), ((5, 5), None, (4, 4)), seed=12, theta=0.8)
    nx, ny, nz = wl["shape"]
    wl["sources"] = [dict(comp=1, box=(nx // 3, nx // 3 + 1, 0, ny, nz // 4, nz // 2), amplitude=2.0,
                          waveform="mod_gauss", freq=3e14, t0=1.5e-15, tw=6e-16)]
    obj = (1, (2 * nx // 3, 2 * nx // 3 + 1, 0, ny, 0, nz), 2.5e14)
    print(f"case: adjoint classes vs maps, {wl['shape']}, {dtype}", flush=True)
    F1, gl1, gs1 = gpu_adjoint(wl, obj, 30, 6, dtype, edge_classes=True)
    F0, gl0, gs0 = gpu_adjoint(wl, obj, 30, 6, dtype, edge_classes=False)
    assert F1 == F0
    assert np.array_equal(gl1, gl0) and np.array_equal(gs1, gs0)
