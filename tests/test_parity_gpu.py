"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: relative L2 <= 1e-12 per field group for the FP64 path, <= 1e-5
for the FP32 path (both started from the same FP32-rounded inputs), after the
stated number of steps.  Grids are chosen to span several column tiles (64
wide, 4-8 rows, 8-64 planes: the sweeps pick the z length at launch from the
grid size) with ragged tails, degenerate axes and every boundary combination.
"""
import numpy as np
import pytest

from paper_2305_13419_amd import workloads
from tests.helpers import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def check(wl, steps, dtype, **kw):
    print(f"case: {wl['name']} pml={wl['pml']} steps={steps} dtype={dtype}", flush=True)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    g = run_gpu(wl, steps, dtype, **kw)
    o = run_oracle(wl, steps, npdt)
    res = compare(g, o)
    print("  rel-L2:", {k: f"{v:.2e}" for k, v in res.items()}, flush=True)
    for k, v in res.items():
        assert v <= TOL[dtype], (k, v)
    return res


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_periodic_ragged(dtype, theta):
    wl = workloads.random_medium((70, 37, 45), seed=3, theta=theta)
    check(wl, 25, dtype)


PML_CASES = [((6, 5), None, None), (None, (4, 4), None), (None, None, (3, 6)),
             ((5, 5), (4, 3), (6, 4)), ((0, 0), None, (0, 0))]


@pytest.mark.parametrize("pml", PML_CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cpml_sources_probes(pml, dtype):
    wl = workloads.random_medium((66, 21, 40), seed=5, pml=pml)
    wl["sources"] = [
        dict(comp=1, box=(30, 31, 0, 21, 10, 30), amplitude=2.0, waveform="mod_gauss", freq=3e14, t0=2e-15, tw=8e-16),
        dict(comp=2, box=(10, 50, 5, 6, 20, 21), amplitude=-1.0, waveform="sin", freq=1e14),
        dict(comp=0, box=(12, 14, 7, 9, 3, 5), amplitude=0.5, waveform="gauss", t0=1e-15, tw=5e-16),
    ]
    wl["probes"] = [dict(comp=1, box=(40, 41, 0, 21, 0, 40), freqs=(3e14, 1e14)),
                    dict(comp=0, box=(20, 21, 10, 11, 15, 16), freqs=(2e14,)),
                    dict(comp=2, box=(0, 66, 0, 21, 0, 40))]
    check(wl, 30, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_overlapping_sources(dtype):
    """Boxes that overlap on one component add in source order (the sweep adds every source whose
    box holds an edge to the new E there, in source order); a second component overlaps them too,
    and a one-cell box sits inside two others."""
    wl = workloads.random_medium((40, 18, 22), seed=11, pml=(None, (3, 3), None))
    wl["sources"] = [
        dict(comp=1, box=(5, 30, 2, 14, 4, 18), amplitude=1.5, waveform="sin", freq=2e14),
        dict(comp=1, box=(10, 12, 0, 18, 0, 22), amplitude=-0.7, waveform="mod_gauss", freq=3e14, t0=2e-15, tw=8e-16),
        dict(comp=2, box=(8, 20, 6, 9, 3, 12), amplitude=0.9, waveform="gauss", t0=1e-15, tw=5e-16),
        dict(comp=1, box=(11, 12, 5, 6, 10, 11), amplitude=3.0, waveform="sin", freq=1e14),
    ]
    wl["probes"] = [dict(comp=1, box=(11, 12, 0, 18, 0, 22), freqs=(2e14,))]
    check(wl, 20, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mid_size_grid(dtype):
    """8.4 M cells: the launch rule picks 16-plane tiles for the FP32 sweeps and the FP64 E pass
    and 32-plane tiles for the FP64 H pass, which the small grids (8 planes) do not reach."""
    wl = workloads.random_medium((256, 128, 256), seed=23, pml=((4, 4), None, (6, 6)))
    check(wl, 3, dtype)


@pytest.mark.parametrize("shape", [(1, 1, 96), (80, 1, 1), (1, 70, 1), (1, 1, 1), (3, 5, 2), (130, 9, 1)])
def test_degenerate_axes(shape):
    wl = workloads.random_medium(shape, seed=9)
    check(wl, 40, torch.float64)


def test_chunked_stepping_matches_single_call():
    wl = workloads.random_medium((40, 12, 36), seed=11, pml=((5, 5), None, None))
    wl["probes"] = [dict(comp=1, box=(20, 21, 0, 12, 0, 36), freqs=(1e14,))]
    a = run_gpu(wl, 24, torch.float64)
    b = run_gpu(wl, 24, torch.float64, chunks=[1, 7, 16])
    for x, y in zip(a[:3], b[:3]):
        for p, q in zip(x, y):
            assert np.array_equal(p, q)
    assert np.array_equal(a[3][0][0], b[3][0][0])


def test_determinism_bitwise():
    wl = workloads.random_medium((70, 37, 45), seed=13, pml=(None, (3, 3), None))
    a = run_gpu(wl, 20, torch.float64)
    b = run_gpu(wl, 20, torch.float64)
    for x, y in zip(a[:3], b[:3]):
        for p, q in zip(x, y):
            assert np.array_equal(p, q)


def test_energy_matches_oracle_and_identity():
    """GPU energy functional equals the oracle's; lossless periodic runs conserve it."""
    from oracle.oracle import OracleSim
    from paper_2305_13419_amd import Simulation
    from tests.helpers import MU0

    wl = workloads.random_medium((34, 20, 36), seed=17, sigma_max=0.0)
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], 1.0, torch.float64)
    sim.set_materials(*wl["maps"])
    E, H, J = wl["fields"]
    sim.set_fields(E, H, J)
    o = OracleSim(wl["shape"], wl["spacing"], wl["dt"], 1.0)
    o.set_materials(*wl["maps"])
    o.set_fields(E, [h * MU0 for h in H], J)
    W0, bad = sim.energy()
    assert bad == 0
    assert abs(W0 / o.energy() - 1) < 1e-12
    sim.step(50)
    o.step(50)
    W1, _ = sim.energy()
    assert abs(W1 / o.energy() - 1) < 1e-12
    assert abs(W1 / W0 - 1) < 1e-12


def test_save_load_state_roundtrip():
    from paper_2305_13419_amd import Simulation

    wl = workloads.random_medium((40, 16, 40), seed=19, pml=((4, 4), None, (4, 4)))
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], 1.0, torch.float64, wl["pml"])
    sim.set_materials(*wl["maps"])
    sim.set_fields(*wl["fields"])
    sim.step(10)
    snap = sim.save_state()
    n = sim.step_index
    sim.step(15)
    ref = [t.clone() for t in sim.E + sim.H + sim.J]
    sim.load_state(snap)
    sim.set_step(n)
    sim.step(15)
    for a, b in zip(ref, sim.E + sim.H + sim.J):
        assert torch.equal(a, b)


def test_unstable_dt_rejected():
    from paper_2305_13419_amd import Simulation
    from paper_2305_13419_amd._lib import TFL_E_UNSTABLE, TflError

    wl = workloads.random_medium((16, 8, 8), seed=1)
    ell_max = wl["maps"][2].max()
    dt = workloads.courant_dt(wl["spacing"], ell_max, 1.02)
    sim = Simulation(wl["shape"], wl["spacing"], dt, 1.0, torch.float64)
    with pytest.raises(TflError) as ei:
        sim.set_materials(*wl["maps"])
    assert ei.value.code == TFL_E_UNSTABLE
    bad = [m.copy() for m in wl["maps"]]
    bad[0][0, 0, 0] = 0.0
    sim2 = Simulation(wl["shape"], wl["spacing"], wl["dt"], 1.0, torch.float64)
    with pytest.raises(TflError):
        sim2.set_materials(*bad)
    bad[0][0, 0, 0] = np.nan
    with pytest.raises(TflError):
        sim2.set_materials(*bad)


@pytest.mark.parametrize("dtype,pml,fused,every,plant", [
    (torch.float64, (None, None, None), True, 1, "E"),
    (torch.float32, ((4, 4), None, (3, 3)), False, 4, "H"),
    (torch.float64, ((4, 4), (2, 2), None), True, 3, "J"),
])
def test_nonfinite_check_reports_planted_value(dtype, pml, fused, every, plant):
    """A NaN or Inf written into the state is counted by tfl_energy and, with the step check on, makes
    tfl_step fail with TFL_E_NONFINITE naming the first checked step; a clean run with the check on
    passes and equals the run without it bit for bit."""
    import math

    from paper_2305_13419_amd import Simulation, _lib as L
    wl = workloads.random_medium((40, 12, 14), seed=5, pml=pml)

    def make():
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"], fused=fused)
        sim.set_materials(*wl["maps"])
        sim.set_fields(*wl["fields"])
        return sim

    clean, checked = make(), make()
    checked.set_nonfinite_check(1)
    clean.step(7)
    checked.step(7)
    for a, b in zip(clean.E + clean.H + clean.J, checked.E + checked.H + checked.J):
        assert torch.equal(a, b)
    assert checked.energy()[1] == 0

    sim = make()
    grp = {"E": sim.E, "H": sim.H, "J": sim.J}[plant]
    if plant == "J":  # Js is read only on superconducting edges: plant where one is
        ell = np.asarray(wl["maps"][2])
        k, j, i = np.argwhere(ell > 0)[0]
        grp[2][k, j, i] = math.inf
    else:
        grp[1][5, 6, 20] = math.nan
    assert sim.energy()[1] >= 1
    sim.set_nonfinite_check(every)
    with pytest.raises(L.TflError) as err:
        sim.step(2 * every)
    assert err.value.code == L.TFL_E_NONFINITE
    assert f"first seen after step {every}" in str(err.value), str(err.value)
    assert sim.step_index == 2 * every  # every step of the call was taken
    sim.set_nonfinite_check(0)
    sim.step(1)  # off again: no error
