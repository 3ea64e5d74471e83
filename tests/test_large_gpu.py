"""The large mixed-precision workload (1024 x 512 x 256 = 134M cells) at full size:
the first steps against the oracle (it can afford a few steps of this grid)."""
import numpy as np
import pytest

from paper_2305_13419_amd import workloads
from tests.helpers import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_large_grid_first_steps_match_oracle():
    wl = workloads.large_mixed_grid()
    steps = 3
    for dtype, npdt, tol in ((torch.float32, np.float32, 1e-5), (torch.float64, np.float64, 1e-12)):
        print(f"case: {wl['name']} {steps} steps {dtype}", flush=True)
        g = run_gpu(wl, steps, dtype)
        torch.cuda.empty_cache()
        o = run_oracle(wl, steps, npdt)
        r = compare(g, o)
        print(f"  rel-L2 vs oracle {r}", flush=True)
        assert max(r.values()) <= tol
        del g, o


def test_roofline_grid_full_size_matches_oracle():
    """The 256^3 roofline grid in the configuration bench.py times (fused sweep with edge classes,
    nontemporal stores, FP32 on 256-cell rows): 4 steps against the oracle over every cell."""
    wl = workloads.roofline_grid(256)
    steps = 4
    for dtype, npdt, tol in ((torch.float64, np.float64, 1e-12), (torch.float32, np.float32, 1e-5)):
        print(f"case: {wl['name']} {steps} steps {dtype}", flush=True)
        g = run_gpu(wl, steps, dtype)
        torch.cuda.empty_cache()
        o = run_oracle(wl, steps, npdt)
        r = compare(g, o)
        print(f"  rel-L2 vs oracle {r}", flush=True)
        assert max(r.values()) <= tol
        del g, o
