"""Build the HVOX HIP library (libhvox.so) for gfx950 with hipcc.

Every call compiles from source.  The kernels are compiled with packed FP32
instructions disabled and hardware float atomics enabled; the planner is
compiled with floating-point contraction off (its partition decisions must
be plain IEEE arithmetic)."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libhvox.so")
ARCH = os.environ.get("HVOX_OFFLOAD_ARCH", "gfx950")

COMMON = ["-std=c++17", "-O3", "-fPIC", "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="hvox_build_") as tmp:
        objs = []
        for src, extra in (("kernels.hip", DEVICE), ("api.cpp", ["-x", "hip"] + DEVICE),
                           ("planner.cpp", ["-ffp-contract=off"])):
            obj = os.path.join(tmp, src + ".o")
            _run([hipcc] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj], verbose)
            objs.append(obj)
        out_tmp = LIB + ".tmp"
        _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", out_tmp] + objs, verbose)
        os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
