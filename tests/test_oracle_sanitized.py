"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize_driver.c calls every oracle entry point once on an 864-particle
jittered fcc lattice (including a neighbour query whose output buffer is too
small, and runs under both rebuild rules) and checks that the calls agree with
each other.  Any out-of-bounds access, use after free, leak, signed overflow or
other undefined behaviour ends the run with a non-zero status.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "mdref.c"), os.path.join(HERE, "sanitize_driver.c"), "-lm", "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("sanitizer runtime not installed")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stderr[-4000:]
    assert res.stdout.strip() == "OK"
