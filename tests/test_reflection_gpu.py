"""The paper's reflection experiment (Sec. 4.2, Eqs. beta, Ref, beta_cases) on the GPU path in FP64: the
4480-cell line of 20 nm cells (vacuum below 7 um, a superconductor with lambda_L = 100 nm and sigma = 0 or
1e4 S/m above, CPML outside both ends), the soft Gaussian pulse, 15 800 steps.  The fields and the probe
series of all three runs (the all-vacuum one gives the incident wave) match the oracle: the fields
after 450 steps, when the pulse has just met the interface and the fields and Js are near their largest
(later the pulse leaves through the CPML and the lossy superconductor absorbs what entered, so the
fields left in the line are orders of magnitude smaller and a relative L2 of them would measure the
rounding of the peak against a residue), and the series over the whole run.  The
reflection coefficient R(f) = |E_r / E_i|^2 computed from the GPU series matches the scheme's own
frequency-domain reflection bin by bin, as the oracle's does."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from tests.helpers import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

D, NDOM, NPML, STEPS, MID = 20e-9, 4480, 32, 15800, 450
N = NDOM + 2 * NPML
DT = 0.95 * D / cf.C0
TW = 0.5e-15  # the pulse width reading of the oracle pin: covers 0-1000 THz
I_SRC, I_OBS, I_SC = NPML + 5, NPML + 340, NPML + 350
ELL = 1 / (100e-9) ** 2


def workload(sig, sc):
    shp = (1, 1, N)
    s, l = np.zeros(shp), np.zeros(shp)
    if sc:
        s[..., I_SC:] = sig
        l[..., I_SC:] = ELL
    return dict(name=f"reflection line sigma={sig:g} sc={sc}", shape=(N, 1, 1), spacing=(D, 1.0, 1.0), dt=DT,
                theta=1.0, pml=((NPML, NPML), None, None), maps=(np.ones(shp), s, l), fields=None,
                sources=[dict(comp=1, box=(I_SRC, I_SRC + 1, 0, 1, 0, 1), amplitude=1.0, waveform="gauss",
                              freq=0.0, t0=4 * TW, tw=TW)],
                probes=[dict(comp=1, box=(I_OBS, I_OBS + 1, 0, 1, 0, 1))], steps=STEPS)


def test_reflection_experiment_matches_oracle_and_the_discrete_reflection():
    series = {}
    for key, (sig, sc) in {"vacuum": (0.0, False), 0.0: (0.0, True), 1e4: (1e4, True)}.items():
        wl = workload(sig, sc)
        # the fields while the pulse is at the interface, then the probe series of the whole run
        print(f"case: {wl['name']}, fields after {MID} steps, GPU FP64 and oracle", flush=True)
        r = compare(run_gpu(wl, MID, torch.float64), run_oracle(wl, MID))
        print(f"  rel-L2 vs oracle: {r}", flush=True)
        assert max(r.values()) <= 1e-12, r
        print(f"case: {wl['name']}, probe series over {STEPS} steps", flush=True)
        g = run_gpu(wl, STEPS, torch.float64, probe_cap=STEPS + 1)
        o = run_oracle(wl, STEPS, probe_cap=STEPS + 1)
        r = compare(g, o)["probe0"]
        print(f"  series rel-L2 vs oracle: {r:.2e}", flush=True)
        assert r <= 1e-12
        series[key] = (np.asarray(g[3][0][0]), np.asarray(o[3][0][0]))
    f = np.fft.rfftfreq(series["vacuum"][0].size, DT)
    band = np.abs(np.fft.rfft(series["vacuum"][1])) > 1e-3 * np.abs(np.fft.rfft(series["vacuum"][1])).max()
    band[0] = False
    for sig, tol in ((1e4, 1e-4), (0.0, 1e-2)):
        R = []
        for side in (0, 1):  # 0: GPU, 1: oracle
            Fi = np.fft.rfft(series["vacuum"][side])
            Fr = np.fft.rfft(series[sig][side] - series["vacuum"][side])  # reflected = total - incident
            R.append(np.abs(Fr[band]) ** 2 / np.abs(Fi[band]) ** 2)
        sc = (1.0, sig, ELL)
        Rd = np.array([abs(cf.discrete_reflection(x, D, DT, 1.0, (1.0, 0.0, 0.0), sc, m0=sc)) ** 2 for x in f[band]])
        print(f"sigma {sig:g}: max |R_gpu - R_oracle| {np.max(np.abs(R[0] - R[1])):.2e}, "
              f"max |R_gpu - R_discrete| {np.max(np.abs(R[0] - Rd)):.2e}", flush=True)
        assert np.max(np.abs(R[0] - R[1])) <= 1e-10
        assert np.max(np.abs(R[0] - Rd)) <= tol
