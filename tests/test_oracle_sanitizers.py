"""The oracle (C) under AddressSanitizer and UndefinedBehaviorSanitizer, on
random, special and extreme-scale matrices, every flag combination.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-std=c99", "-D_DEFAULT_SOURCE", "-pthread", "-o", exe,
           os.path.join(ORC, "sanitize_driver.c"), os.path.join(ORC, "syev3_oracle.c"),
           os.path.join(ORC, "jacobi_cyclic.c"), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "0 bad results" in p.stdout
