"""Build the HIP library libnep_hip.so (gfx950) in-tree.

Usage:  python -m paper_2305_08140_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["nep_kernels.hip", "nep_build.hip", "nep_defects.hip", "nep_wide.hip", "nep_thermostat.hip",
           "nep_abi.hip"]
LIB = os.path.join(HERE, "libnep_hip.so")
HOSTMATH_LIB = os.path.join(HERE, "libnep_hostmath.so")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay disabled: plain FMA only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # scalar helpers compiled for the host, for the CPU unit tests
    tmp = HOSTMATH_LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + [os.path.join(HERE, "csrc", "nep_hostmath.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, HOSTMATH_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
