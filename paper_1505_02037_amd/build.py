"""Build the HIP library (gfx950) into paper_1505_02037_amd/liblbnr.so.

Flags that matter for the numerics: -ffp-contract=off (no fused multiply-add,
so every product and sum rounds as written) and no fast-math.  Packed FP32
instructions are disabled for all device code.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbnr.so")
PROBE_LIB = os.path.join(HERE, "libhbmprobe.so")
SOURCES = ["lb_api.hip", "lb_fp64.hip", "lb_fp32.hip", "lb_fused.hip", "lb_serve.hip", "lb_state.hip"]
ARCH = os.environ.get("LBNR_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-shared", "-std=c++17",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]


# roctx ranges around the library calls (visible in a profiler's marker trace)
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def build(verbose: bool = False, extra=None) -> str:
    cmd = ["/opt/rocm/bin/hipcc", *FLAGS, *(extra or []),
           *[os.path.join(CSRC, s) for s in SOURCES], *LIBS, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = ["/opt/rocm/bin/hipcc", *FLAGS, os.path.join(CSRC, "hbm_probe.hip"), "-o", PROBE_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, extra=sys.argv[1:]))
