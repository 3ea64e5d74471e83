"""The allocation-free energy entry point (tfl_energy_noalloc) against tfl_energy through the C ABI:
two calls in a row, the second on a smaller grid, each equal to tfl_energy's results bit for bit (the
same reduction order), including a non-finite count."""
import ctypes
import math

import numpy as np
import pytest

from paper_2305_13419_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def energy_both(sim):
    from paper_2305_13419_amd import _lib as L
    out = torch.full((2,), -1.0, dtype=torch.float64, device=sim.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.call("tfl_energy_noalloc", sim._h, ctypes.c_void_p(out.data_ptr()), stream, handle=sim._h)
    torch.cuda.synchronize()
    w_na, bad_na = out.cpu().tolist()
    w, bad = sim.energy()
    return (w_na, bad_na), (w, bad)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_energy_noalloc_equals_energy(dtype):
    from paper_2305_13419_amd import Simulation
    results = []
    for shape, pml, plant in (((72, 40, 36), (None, None, None), False), ((20, 9, 7), ((3, 3), None, None), True)):
        wl = workloads.random_medium(shape, seed=23, pml=pml)
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"])
        sim.set_materials(*wl["maps"])
        sim.set_fields(*wl["fields"])
        sim.step(5)
        if plant:
            sim.E[0][3, 4, 5] = math.nan
            sim.H[2][1, 2, 3] = math.inf
        (w_na, bad_na), (w, bad) = energy_both(sim)
        print(f"{dtype} {shape}: noalloc W {w_na!r} bad {bad_na}; tfl_energy W {w!r} bad {bad}", flush=True)
        if plant:
            assert bad == 2 and bad_na == 2.0
            assert math.isnan(w) and math.isnan(w_na)
        else:
            assert bad == 0 and bad_na == 0.0
            assert w_na == w and w > 0
        results.append(w_na)
        sim.close()
    assert results[0] != results[1] or math.isnan(results[1])


def test_energy_noalloc_rejects_bad_output():
    from paper_2305_13419_amd import Simulation, _lib as L
    wl = workloads.random_medium((16, 8, 8), seed=3)
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], torch.float64)
    rc = L.lib().tfl_energy_noalloc(sim._h, None, None)
    assert rc == L.TFL_E_STATE  # no materials yet
    sim.set_materials(*wl["maps"])
    assert L.lib().tfl_energy_noalloc(sim._h, None, None) == L.TFL_E_INVAL
    assert L.lib().tfl_energy_noalloc(sim._h, ctypes.c_void_p(0x1004), None) == L.TFL_E_INVAL
    sim.close()
