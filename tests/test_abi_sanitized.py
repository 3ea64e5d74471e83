"""The host code of the C ABI built with AddressSanitizer and UndefinedBehaviorSanitizer (host pass
only; the device code is built as usual) passes the host-side ABI checks of tests/test_abi_cpu.py
(creation, validation of bad configurations, buffer sizes, call order, the fused-buffer and edge-class
layouts) without a report.  Runs on the host: no call reaches the GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_13419_amd", "csrc")


@pytest.mark.slow
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2305_13419_amd import _build
    lib = str(tmp_path / "libtfl_san.so")
    srcs = [os.path.join(CSRC, s) for s in _build.SOURCES if os.path.exists(os.path.join(CSRC, s))]
    flags = [f for f in _build.HIPCC_FLAGS if f != "-O3"] + ["-O1"]
    # each sanitizer flag applies to the host pass only
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    subprocess.check_call([hipcc] + flags + san + ["-o", lib] + srcs, stdout=subprocess.DEVNULL,
                          stderr=subprocess.DEVNULL, timeout=1200)
    preload = []
    for rt in ("libasan.so", "libubsan.so"):
        p = subprocess.check_output(["gcc", f"-print-file-name={rt}"], text=True).strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"{rt} not found")
        preload.append(p)
    env = dict(os.environ, TFL_LIB=lib, LD_PRELOAD=":".join(preload), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_cpu.py"), "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in report and "runtime error" not in report, report
