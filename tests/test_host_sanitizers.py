"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

libmuca: tests/native/host_sanitize.cpp drives every entry point that runs
without a device over ordinary, degenerate and invalid inputs.  The sanitizers
instrument host code only; the kernels are compiled as usual and never run.
The oracle: its C code, built instrumented, runs every exported function, and
its threaded sweeps run under ThreadSanitizer."""
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


_ORACLE_DRIVE = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
oracle._build.build = lambda force=False: sys.argv[2]
assert oracle.lib()._name == sys.argv[2]
oracle.philox((1, 2, 3, 4), (5, 6))
oracle.reachable(oracle.ISING, 2, 6)
oracle.reachable(oracle.POTTS, 8, 5)
oracle.bruteforce(oracle.POTTS, 3, 3)
oracle.bruteforce_canonical(oracle.ISING, 2, 4, 0.4)
oracle.bruteforce_mag(4, 0.66)
oracle.build_table_mag(6, 0.66, np.linspace(0.0, 3.0, 37))
for model, L, q, beta in ((oracle.ISING, 6, 2, 0.0), (oracle.POTTS, 5, 8, 0.0), (oracle.POTTS, 3, 3, 0.0),
                          (oracle.ISING_MAG, 6, 2, 0.66)):
    r = oracle.OracleRun(model, L, 7, 11, q=q, n_threads=3, beta=beta)
    for _ in range(3):
        r.iterate(20, correct=(model != oracle.ISING_MAG))
    r.production(5, 20)
print("oracle drive ok")
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    """The oracle's C code (muca_oracle.c) built with AddressSanitizer and
    UndefinedBehaviorSanitizer: every function it exports runs once, the
    sampler on Ising, 8- and 3-state Potts and the multimagnetic ensemble
    with several threads, with no report."""
    so = str(tmp_path / "libmuca_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", so, os.path.join(ROOT, "oracle", "muca_oracle.c"), "-lm", "-lpthread"],
                   check=True, capture_output=True, timeout=300)
    pre = [subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
           for n in ("libasan.so", "libubsan.so")]
    if not all(os.path.isabs(p) and os.path.exists(p) for p in pre):
        pytest.skip("sanitizer runtimes not found")
    env = dict(os.environ, LD_PRELOAD=":".join(pre), ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    import sys
    res = subprocess.run([sys.executable, "-c", _ORACLE_DRIVE, ROOT, so], capture_output=True, text=True,
                         timeout=600, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "Sanitizer" not in res.stderr, res.stderr
    assert "oracle drive ok" in res.stdout


_ORACLE_THREADS = r"""
import sys
sys.path.insert(0, sys.argv[1])
import oracle
oracle._build.build = lambda force=False: sys.argv[2]
assert oracle.lib()._name == sys.argv[2]
for model, L, q, beta in ((oracle.ISING, 6, 2, 0.0), (oracle.POTTS, 5, 8, 0.0), (oracle.ISING_MAG, 6, 2, 0.66)):
    r = oracle.OracleRun(model, L, 13, 11, q=q, n_threads=4, beta=beta)
    for _ in range(3):
        r.iterate(20)
    r.production(5, 20)
print("oracle threads ok")
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_threads_are_clean_under_thread_sanitizer(tmp_path):
    """The oracle's sweeps split the chains over threads; built with
    ThreadSanitizer, four threads over 13 chains report no data race."""
    so = str(tmp_path / "libmuca_oracle_tsan.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                    "-fsanitize=thread", "-o", so, os.path.join(ROOT, "oracle", "muca_oracle.c"), "-lm", "-lpthread"],
                   check=True, capture_output=True, timeout=300)
    rt = subprocess.run(["gcc", "-print-file-name=libtsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(rt) and os.path.exists(rt)):
        pytest.skip("thread sanitizer runtime not found")
    env = dict(os.environ, LD_PRELOAD=rt, TSAN_OPTIONS="halt_on_error=1")
    import sys
    res = subprocess.run([sys.executable, "-c", _ORACLE_THREADS, ROOT, so], capture_output=True, text=True,
                         timeout=600, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ThreadSanitizer" not in res.stderr, res.stderr
    assert "oracle threads ok" in res.stdout
