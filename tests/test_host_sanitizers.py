"""The host code of libmuca under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): tests/native/host_sanitize.cpp drives every entry point that runs
without a device over ordinary, degenerate and invalid inputs.  The sanitizers
instrument host code only; the kernels are compiled as usual and never run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1212_3975_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("muca_kernels.hip", "muca_api.cpp", "mlp_kernels.hip", "mlp_api.cpp")]
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_host_entry_points_are_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-o", exe,
           os.path.join(ROOT, "tests", "native", "host_sanitize.cpp"), *SOURCES]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "Sanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr
    assert "failures 0" in res.stdout
