"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver (tests/csrc/oracle_sanitize_driver.c) calls every entry point on
small random inputs, N = 1 .. 2^11, in a build where any out-of-bounds
access, leak, overflow or other undefined behaviour aborts."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
           os.path.join(ROOT, "oracle", "sc_oracle.c"), os.path.join(HERE, "csrc", "oracle_sanitize_driver.c"),
           "-o", str(exe), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]
