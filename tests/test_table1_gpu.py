"""The paper's skin-depth sweep (Sec. 4.1, Table 1) on the GPU (FP64), ten of its twelve rows: the skin
depth measured from the simulated field, z0 / ln(A(0) / A(z0)) with steady-state amplitudes over the
last two of five periods, against the discrete scheme's prediction 1 / Im k (oracle closed form) and
the paper's computed column.  The undamped 100 THz row sits 16 % below the medium's cutoff (119 THz):
the sudden start of the sine excites waves just above the cutoff whose group velocity is near zero and
which stay at the source for tens of periods (the paper's own value there is 0.7 % off the theory), so
that row runs 200 periods and fits the last 50.  The 100 GHz rows take 1.7 M steps and the 25 GHz rows
6.7 M steps each (about 12 and 49 s on one GPU: the 6065-cell line is launch-bound); the two 25 GHz rows
left out (sigma = 0 and 1e4, both 400.010 nm) pass the same check in `bench.py --table1`.  One row per
conductivity (100 THz, five periods) is also compared with the oracle, field by field and sample by
sample."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from paper_2305_13419_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
ELL = 1.0 / (400e-9) ** 2


# every row at 100 GHz and above, and of the 25 GHz rows (6.7 M steps, about 50 s each) the one whose
# skin depth differs from lambda_L (sigma = 1e7: 395 nm); the other two run in `bench.py --table1`
ROWS = [r for r in workloads.TABLE1_ROWS if r[1] >= 1e11 or r[0] == 1e7]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("sigma,freq,paper", ROWS)
def test_table1_row(sigma, freq, paper):
    from paper_2305_13419_amd import Simulation
    theory = float(cf.skin_depth(freq, 1.0, sigma, ELL))
    near_cutoff = sigma == 0.0 and freq == 1e14
    wl = workloads.table1_grid(sigma, freq, theory, periods=200 if near_cutoff else 5)
    discrete = cf.discrete_skin_depth(freq, 10e-9, wl["dt"], 1.0, 1.0, sigma, ELL)
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], 1.0, torch.float64, wl["pml"])
    sim.set_materials(*wl["maps"])
    for s in wl["sources"]:
        sim.add_source(**s)
    pids = [sim.add_probe(p["comp"], p["box"], wl["steps"] + 1) for p in wl["probes"]]
    left = wl["steps"]
    while left > 0:  # a progress line per 500 000 steps (~4 s)
        c = min(left, 500000)
        sim.step(c)
        left -= c
        torch.cuda.synchronize()
        print(f"  {wl['steps'] - left} / {wl['steps']} steps", flush=True)
    a0, a1 = (workloads.steady_amplitude(sim.probe(p)[0], wl["dt"], freq, periods=50 if near_cutoff else 2)
              for p in pids)
    delta = wl["z0"] / np.log(a0 / a1)
    print(f"Table 1 sigma {sigma:g} f {freq:g}: computed {delta * 1e9:.3f} nm, discrete {discrete * 1e9:.3f}, "
          f"theory {theory * 1e9:.3f}, paper computed {paper}  ({wl['steps']} steps)", flush=True)
    sim.close()
    # the steady state of the discrete scheme decays exactly as exp(-|x| Im k) node by node
    assert abs(delta / discrete - 1) < 2e-3


@pytest.mark.parametrize("sigma", [0.0, 1e4, 1e7])
def test_table1_100thz_row_matches_oracle(sigma):
    """The 100 THz row of each conductivity (five periods, 1667 steps on 6065 cells with CPML ends and
    the soft sine at the centre): fields and both probe series of the GPU path against the oracle."""
    from tests.helpers import compare, run_gpu, run_oracle
    theory = float(cf.skin_depth(1e14, 1.0, sigma, ELL))
    wl = workloads.table1_grid(sigma, 1e14, theory)
    g = run_gpu(wl, wl["steps"], torch.float64)
    o = run_oracle(wl, wl["steps"])
    r = compare(g, o)
    print(f"Table 1 sigma {sigma:g} 100 THz, {wl['steps']} steps: rel-L2 vs oracle {r}", flush=True)
    assert max(r.values()) <= 1e-12
