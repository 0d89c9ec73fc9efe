"""The library's host C++ under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no GPU): the planner, the frozen-set builders, argument checks and
the tune-file parser, driven by tests/csrc/host_sanitize_driver.cpp with the
device layer stubbed.  Sanitizers apply to host code only (each -fsanitize
flag goes to the host pass); the device code of the construction's file is
compiled as usual and never launched.  Any out-of-bounds access, leak,
overflow or other undefined behaviour aborts the driver.  (The planner once
sized a stack array for four check-update kinds; with a fifth kind the
driver's plans index past it, which the sanitized driver reports.)"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1204_5882_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("gcc") is None, reason="hipcc not available")
def test_host_code_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "host_sanitized"
    cmd = [HIPCC, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           *[os.path.join(CSRC, f) for f in ("polar_host.cpp", "polar_tune.cpp", "polar_serve.cpp",
                                             "polar_construct.hip")],
           os.path.join(HERE, "csrc", "host_sanitize_driver.cpp"),
           "-o", str(exe), "-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]
