"""The paper's CPW resonator at its own size (Sec. 5: 130 x 1008 x 1280 cells, dx = dy = 1 um,
dz = 50 nm, plus CPML slabs on every face, 196 M cells): the first four steps from seeded random
fields (one round trip of the two-step sweep, which the automatic policy takes here in FP64), with
the film of case 3 (sigma = 6e7 S/m, lambda_L = 100 nm), the two soft sources and the probes,
against the oracle in FP64 (the oracle runs on the host: about 50 GB and a minute per step at this
size)."""
import numpy as np
import pytest

from paper_2305_13419_amd import workloads
from tests.helpers import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_paper_cpw_first_steps_match_oracle():
    wl = workloads.paper_cpw_grid(3, fields="random")
    steps = 4
    print(f"case: {wl['name']} {steps} steps FP64", flush=True)
    g = run_gpu(wl, steps, torch.float64)
    torch.cuda.empty_cache()
    o = run_oracle(wl, steps, np.float64)
    r = compare(g, o)
    print(f"  rel-L2 vs oracle {r}", flush=True)
    assert max(r.values()) <= 1e-12
