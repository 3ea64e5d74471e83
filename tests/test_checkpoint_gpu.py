"""Restart files: a run written by Simulation.save_checkpoint and continued in a fresh simulation by
load_checkpoint gives the fields, currents, CPML variables and probe series / DFTs of the uninterrupted
run bit for bit; a simulation that describes another run refuses the file."""
import numpy as np
import pytest

from paper_2305_13419_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make(wl, dtype, dt=None):
    from paper_2305_13419_amd import Simulation
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"] if dt is None else dt, wl["theta"], dtype, wl["pml"])
    sim.set_materials(*wl["maps"])
    z = [np.zeros(sim.shape3)] * 3
    sim.set_fields(z, z, z)
    for s in wl["sources"]:
        sim.add_source(**s)
    pids = [sim.add_probe(p["comp"], p["box"], 200, [wl["freq"], 0.5 * wl["freq"]]) for p in wl["probes"]]
    return sim, pids


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_restart_file_continues_the_run_bit_for_bit(tmp_path, dtype):
    wl = workloads.cpw_grid(4)  # CPML on x and z, film, two soft sources, two probes
    path = str(tmp_path / "run.npz")
    print(f"case: restart file, {wl['name']}, {dtype}, 37 + 40 steps", flush=True)
    a, pa = make(wl, dtype)
    a.step(37)
    a.save_checkpoint(path)
    a.step(40)
    b, pb = make(wl, dtype)
    b.load_checkpoint(path)
    assert b.step_index == 37
    b.step(40)
    torch.cuda.synchronize()
    assert a.step_index == b.step_index == 77
    for x, y in zip(a.E + a.H + a.J, b.E + b.H + b.J):
        assert torch.equal(x, y)
    assert torch.equal(a.save_state(), b.save_state())  # the CPML variables too
    for p, q in zip(pa, pb):
        sa, da = a.probe(p)
        sb, db = b.probe(q)
        assert np.array_equal(sa, sb) and np.array_equal(da, db)
    c, _ = make(wl, dtype, dt=0.9 * wl["dt"])
    with pytest.raises(ValueError, match="dt"):
        c.load_checkpoint(path)
    for s in (a, b, c):
        s.close()
