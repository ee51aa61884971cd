"""Build the gfx950 library libmpc355.so in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpc355.so")
SOURCES = [os.path.join(HERE, "csrc", "mpc_kernels.hip"),
           os.path.join(HERE, "csrc", "mpc_probe.hip"),
           os.path.join(HERE, "csrc", "mpc_capi.cpp")]

# -ffp-contract=off: every written floating-point operation is one IEEE
# operation (fma() only where the streaming rule asks for it), so FP64 results
# follow the operation order documented in the sources.  Packed FP32 ops are
# switched off for the device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, *inc, "-x", "hip", *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
