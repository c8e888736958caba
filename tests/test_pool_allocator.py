"""The server's device-pool allocator (host bookkeeping), built with g++ and
checked against a byte-map model over random alloc/release sequences, under
AddressSanitizer and UndefinedBehaviorSanitizer.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pool_allocator_against_a_byte_map(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "pool_driver")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined",
                           "-I", os.path.join(ROOT, "paper_1806_06698_amd", "csrc"),
                           os.path.join(ROOT, "tests", "pool_driver.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "pool ok" in p.stdout


def test_pool_allocator_is_exception_safe(tmp_path):
    """A std::bad_alloc from the free list's node allocation (host memory
    exhausted) leaves the allocator unchanged: no range is lost and the byte
    count stays right, so the server can report SYEV3_E_NOMEM and go on."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "pool_fail_driver")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined",
                           "-I", os.path.join(ROOT, "paper_1806_06698_amd", "csrc"),
                           os.path.join(ROOT, "tests", "pool_fail_driver.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "pool exception-safe" in p.stdout
