"""The benchmark's host side: one GPU only, and the HBM traffic it reports comes from the committed
rocprofv3 counter summary of the kernels as they are (a change of the forward kernels' code turns
the figure off until the counters are taken again)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_traffic_matches_the_kernels():
    """The profile's TRAFFIC lines were taken from the current kernels: both precisions of the
    dominant two-step sweep and the one-step sweeps have a figure."""
    for dt in ("f64", "f32"):
        for k in ("two_step_kernel", "fused_step_kernel", "fused_step_kernel_maps", "e_pass_kernel"):
            v = bench.measured_traffic(dt, k)
            assert v is not None and v > 1e8, (dt, k, v)


def test_traffic_is_withheld_for_changed_code(monkeypatch):
    monkeypatch.setattr(bench, "kernel_code_hash", lambda: "0000000000000000")
    assert bench.measured_traffic("f64", "two_step_kernel") is None
