"""Ringdown fit: the NumPy reference recovers synthetic damped modes exactly, and
the library's GPU fit (normal equations on the device) matches it."""
import numpy as np
import pytest

from oracle.ringdown import lp_fit


def synth(n, dt, modes, phase=(0.3, 1.1)):
    t = np.arange(n) * dt
    return sum(A * np.exp(-al * t) * np.cos(2 * np.pi * f * t + ph) for (A, f, al), ph in zip(modes, phase))


@pytest.mark.parametrize("modes", [[(1.0, 0.97e12, 0.97e12 * np.pi / 316)],
                                   [(1.0, 0.97e12, 0.97e12 * np.pi / 316), (0.4, 2.1e12, 2.1e12 * np.pi / 50)]])
def test_reference_fit_recovers_modes(modes):
    dt = 5.2e-16
    decim = 60  # ~32 samples per period at 1 THz
    x = synth(200000, dt, modes)
    r = lp_fit(x, 1000, 2000, decim, 2 * len(modes) + 2, dt, f_hint=modes[0][1])
    f, al = modes[0][1], modes[0][2]
    assert abs(r["f0"] / f - 1) < 1e-10
    assert abs(r["alpha"] / al - 1) < 1e-8
    assert abs(r["Q"] / (np.pi * f / al) - 1) < 1e-8


@pytest.mark.gpu
@pytest.mark.parametrize("order", [4, 0])
def test_gpu_fit_matches_reference(order):
    torch = pytest.importorskip("torch")
    from paper_2305_13419_amd import Simulation
    dt = 5.2e-16
    sim = Simulation((8, 4, 4), (0.5e-6,) * 3, dt, 1.0, torch.float64)
    one = np.ones((4, 4, 8))
    sim.set_materials(one, 0 * one, 0 * one)
    n = 200000
    pid = sim.add_probe(0, (0, 1, 0, 1, 0, 1), n)
    modes = [(1.0, 0.97e12, 0.97e12 * np.pi / 316), (0.4, 2.1e12, 2.1e12 * np.pi / 50)]
    if order == 0:  # order 8: four modes keep the normal equations full rank
        modes += [(0.2, 3.3e12, 3.3e12 * np.pi / 30), (0.1, 4.0e12, 4.0e12 * np.pi / 80)]
    x = synth(n, dt, modes, phase=(0.3, 1.1, 2.0, 0.7))
    sim._probes[pid][0].copy_(torch.tensor(x, device="cuda"))
    g = sim.ringdown_fit(pid, 1000, 2000, 60, order, f_hint=0.97e12)
    r = lp_fit(x, 1000, 2000, 60, g["order"], dt, f_hint=0.97e12)
    assert g["order"] == (4 if order == 4 else 8)  # auto order = numerical rank = 2 x modes
    # the device forms the normal equations (condition number squared): 1e-7 on the damping
    assert abs(g["f0"] / r["f0"] - 1) < 1e-10 and abs(g["alpha"] / r["alpha"] - 1) < 1e-7
    assert abs(g["Q"] / 316 - 1) < 1e-7
