"""The CPU reference under AddressSanitizer and UndefinedBehaviorSanitizer.

A C driver (tests/oracle_sanitize_driver.c) runs every curvature model, both
collision operators, walls with wetting, the bubble model and the frozen mode
on small lattices, reads every output, writes the distributions back and
checks mass conservation; any invalid access, leak or undefined behaviour
fails the run. Host code only: the GPU library is not involved.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_sanitize")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", ORACLE, DRIVER, os.path.join(ORACLE, "fslbm_oracle.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
