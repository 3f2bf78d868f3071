"""Builds libmuca.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libmuca.so")
SOURCES = [os.path.join(CSRC, f) for f in ("muca_kernels.hip", "muca_api.cpp", "muca_static.hip", "mlp_kernels.hip",
                                           "mlp_api.cpp")]
HEADERS = [os.path.join(CSRC, "muca_device.h"), os.path.join(CSRC, "mlp_device.h"), os.path.join(INCLUDE, "muca.h")]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# Host code keeps IEEE double semantics (no contraction, no fast-math) because
# the weight recursion and the acceptance tables are reproduced bit for bit.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", INCLUDE,
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compiles every source.  force=False skips the build when the library
    is newer than all sources."""
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(s) <= t for s in SOURCES + HEADERS):
            return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose="-v" in sys.argv))
