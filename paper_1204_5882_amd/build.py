"""Build libpolar.so for gfx950 with hipcc (cross-compiles without a GPU).

    python -m paper_1204_5882_amd.build

Each translation unit (host code, common device code, and one unit per
decoder variant under csrc/variants) is compiled to an object in parallel,
then linked into paper_1204_5882_amd/libpolar.so next to this file.  The
device assembly of every unit is kept in _build/ (for the ISA checks in the
tests).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
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

SOURCES = ["sc_device.hip", "polar_host.cpp", "polar_tune.cpp", "polar_serve.cpp", "polar_static.hip",
           "polar_fer.hip", "polar_construct.hip", "polar_scl.hip"] + sorted(
    os.path.relpath(f, CSRC) for f in glob.glob(os.path.join(CSRC, "variants", "*.hip")))

# Device code runs with the IEEE mode bit off: min/max then need no NaN
# quieting, so the min-sum check update is one v_min_f32 with |.| modifiers.
# LLRs are finite throughout (no NaN is produced or tested).
DEVICE_ONLY = ["-mno-amdgpu-ieee", "-fno-honor-nans"]


LLVM_BIN = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin")


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"{what} failed")
    return r.stdout


def _dump_isa(obj: str, name: str) -> None:
    """Disassembly and kernel metadata of the gfx950 code object embedded in
    obj, written to _build/<name>.gfx950.isa for the ISA checks."""
    tool = lambda t: os.path.join(LLVM_BIN, t)
    fatbin = os.path.join(BUILD_DIR, name + ".fatbin")
    co = os.path.join(BUILD_DIR, name + ".gfx950.co")
    _run([tool("llvm-objcopy"), "--dump-section", f".hip_fatbin={fatbin}", obj], f"fatbin of {name}")
    _run([tool("clang-offload-bundler"), "--unbundle", "--type=o", f"--input={fatbin}",
          f"--targets=hipv4-amdgcn-amd-amdhsa--{ARCH}", f"--output={co}"], f"unbundle {name}")
    text = _run([tool("llvm-objdump"), "-d", f"--mcpu={ARCH}", co], f"disassemble {name}")
    notes = _run([tool("llvm-readelf"), "--notes", co], f"notes of {name}")
    with open(os.path.join(BUILD_DIR, name + f".{ARCH}.isa"), "w") as f:
        f.write(notes)
        f.write(text)


def _compile(src: str) -> str:
    name = os.path.splitext(os.path.basename(src))[0]
    out = os.path.join(BUILD_DIR, name + ".o")
    cmd = [HIPCC, *COMMON]
    if src.endswith(".hip"):
        cmd += DEVICE_ONLY
    cmd += ["-c", os.path.join(CSRC, src), "-o", out]
    _run(cmd, f"hipcc on {src}")
    if src.endswith(".hip"):
        _dump_isa(out, name)
    return out


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    # longest units first
    order = sorted(SOURCES, key=lambda f: ("prune" not in f, not f.endswith(".hip")))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, order))
    tmp = OUT + ".tmp"
    # roctx ranges of the host calls (rocprofv3 --marker-trace)
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
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
