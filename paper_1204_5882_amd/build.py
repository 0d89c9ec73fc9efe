"""Build libpolar.so for gfx950 with hipcc (cross-compiles without a GPU).

    python -m paper_1204_5882_amd.build

Each translation unit is compiled to an object in parallel, then linked into
paper_1204_5882_amd/libpolar.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libpolar.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]

SOURCES = ["sc_device.hip", "polar_host.cpp"]

# Device code runs with the IEEE mode bit off: min/max then need no NaN
# quieting, so the min-sum check update is one v_min_f32 with |.| modifiers.
# LLRs are finite throughout (no NaN is produced or tested).
DEVICE_ONLY = ["-mno-amdgpu-ieee", "-fno-honor-nans"]


ISA_OUT = os.path.join(BUILD_DIR, "sc_device-gfx950.s")


def _compile(src: str) -> str:
    if src == "@isa":
        # device assembly of the kernels, kept for the ISA checks in the tests
        cmd = [HIPCC, *COMMON, *DEVICE_ONLY, "--cuda-device-only", "-S", os.path.join(CSRC, "sc_device.hip"),
               "-o", ISA_OUT]
        out = ISA_OUT
    else:
        out = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        extra = DEVICE_ONLY if src.endswith(".hip") else []
        cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return out


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        objs = list(ex.map(_compile, SOURCES + ["@isa"]))[: len(SOURCES)]
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
