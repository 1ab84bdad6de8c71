"""Builds libgdrr.so (the HIP library behind include/gdrr.h) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgdrr.so")
SOURCES = [os.path.join(HERE, "csrc", "gdrr_api.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", f) for f in ("gdrr_device.h", "gdrr_kernels.h", "gdrr_raytrace.h", "gdrr_denoise.h")] + \
    [os.path.join(ROOT, "include", "gdrr.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed float32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]


# calibration programs behind the benchmark's rooflines (not part of the library): instruction
# issue costs and random-gather throughput
CALIB = ["issue_rate", "gather_rate", "lds_granule"]      # paper_1204_6367_amd/calib/<name>.hip -> <name>


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in DEPS):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_calibration(verbose: bool = False) -> list:
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC", "-munsafe-fp-atomics")]
    built = []
    for name in CALIB:
        exe = os.path.join(HERE, "calib", name)
        cmd = ["hipcc", *flags, os.path.join(HERE, "calib", name + ".hip"), "-o", exe + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(exe + ".tmp", exe)
        built.append(exe)
    return built


if __name__ == "__main__":
    build(verbose=True)
    build_calibration(verbose=True)
    print(LIB)
    sys.exit(0)
