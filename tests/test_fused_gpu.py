"""The fused sweep (H and E updates of a step in one kernel, periodic grids) gives the same
fields, currents and probe series as the two passes, bit for bit, for odd and even step counts."""
import numpy as np
import pytest

from paper_2305_13419_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def run(wl, steps, dtype, fused, chunks=None):
    from paper_2305_13419_amd import Simulation
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"], fused=fused)
    assert (sim.fused_buffer is not None) == fused
    sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
    E, H, J = wl["fields"]
    sim.set_fields([np.asarray(a, dtype=npdt) for a in E], [np.asarray(a, dtype=npdt) for a in H],
                   [np.asarray(a, dtype=npdt) for a in J])
    sim.add_source(comp=1, box=(30, 31, 0, 21, 10, 30), amplitude=2.0, waveform="mod_gauss", freq=3e14,
                   t0=2e-15, tw=8e-16)
    sim.add_source(comp=2, box=(10, 50, 5, 6, 20, 21), amplitude=-1.0, waveform="sin", freq=1e14)
    pid = sim.add_probe(1, (40, 41, 0, 21, 0, 40), steps + 1, [3e14])
    for c in (chunks or [steps]):
        sim.step(c)
    torch.cuda.synchronize()
    out = [t.clone() for t in sim.E + sim.H + sim.J] + [torch.tensor(np.asarray(sim.probe(pid)[0]))]
    sim.close()
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("steps,chunks", [(1, None), (2, None), (7, None), (20, [3, 5, 1, 11])])
def test_fused_equals_two_pass(dtype, steps, chunks):
    wl = workloads.random_medium((66, 21, 40), seed=5)
    print(f"case: fused vs two-pass, {steps} steps in chunks {chunks}, {dtype}", flush=True)
    a = run(wl, steps, dtype, True, chunks)
    b = run(wl, steps, dtype, False, chunks)
    worst = max(float(((x.double() - y.double()).abs().max() / y.double().abs().max().clamp_min(1e-300)))
                for x, y in zip(a, b))
    print(f"  max relative difference {worst:.3e}", flush=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def run_plain(wl, steps, dtype, fused):
    from paper_2305_13419_amd import Simulation
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"], fused=fused)
    assert (sim.fused_buffer is not None) == fused
    sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
    E, H, _ = wl["fields"]
    sim.set_fields([np.asarray(a, dtype=npdt) for a in E], [np.asarray(a, dtype=npdt) for a in H])
    sim.step(steps)
    torch.cuda.synchronize()
    out = [t.clone() for t in sim.E + sim.H + sim.J]
    sim.close()
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(256, 9, 12), (128, 10, 9), (256, 256, 256)])
def test_fused_row_tiles_and_large_grids_equal_two_pass(shape, dtype):
    """FP32 rows of 256 or 128 cells per block when they tile the x extent, and the nontemporal
    stores of grids past the infinity cache (256^3), against the two passes bit for bit."""
    wl = workloads.roofline_grid(shape)
    print(f"case: fused vs two-pass, roofline boxes {shape}, {dtype}, 3 steps", flush=True)
    a = run_plain(wl, 3, dtype, True)
    b = run_plain(wl, 3, dtype, False)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
