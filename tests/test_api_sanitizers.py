"""The C API's argument validation (syev3_api.cpp) under AddressSanitizer
and UndefinedBehaviorSanitizer, host code only: tests/api_args_driver.cpp
compiles the API source with recording stubs in place of the kernel
launchers and makes randomized calls of every entry point, including sizes
at the ends of int64.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmp_path, api_dir, name):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", api_dir,
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1806_06698_amd", "csrc"),
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", exe, os.path.join(ROOT, "tests", "api_args_driver.cpp")]
    subprocess.check_call(cmd)
    return exe


def _run(exe, cases):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, str(cases)], capture_output=True, text=True, timeout=600,
                          env=env)


def _need_toolchain():
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/hip"):
        pytest.skip("g++ or the HIP headers not available")


def test_api_argument_checks_are_clean_and_match_the_documented_rules(tmp_path):
    _need_toolchain()
    exe = _build(tmp_path, os.path.join(ROOT, "paper_1806_06698_amd", "csrc"), "api_args")
    p = _run(exe, 300_000)
    assert p.returncode == 0, p.stdout + p.stderr
    assert ", 0 failures" in p.stdout
    print(p.stdout.strip())


def test_the_driver_catches_a_missing_alias_check(tmp_path):
    """A copy of the API source with the output-overlap test removed must
    fail the driver (the driver is not vacuous)."""
    _need_toolchain()
    src = open(os.path.join(ROOT, "paper_1806_06698_amd", "csrc", "syev3_api.cpp")).read()
    old = "  if (overlap(ra, rl) || (!inplace && overlap(ra, rv)) || overlap(rl, rv))"
    assert src.count(old) == 1
    mut = tmp_path / "mutant"
    mut.mkdir()
    (mut / "syev3_api.cpp").write_text(src.replace(old, "  if (false && overlap(ra, rl))"))
    exe = _build(tmp_path, str(mut), "api_args_mutant")
    p = _run(exe, 50_000)
    assert p.returncode != 0 and "invalid call accepted" in p.stderr


def test_the_driver_catches_a_missing_cross_segment_alias_check(tmp_path):
    """The same for the segment call: with its check of inputs against other
    segments' outputs removed, the driver must report an accepted call that
    the documented rules forbid."""
    _need_toolchain()
    src = open(os.path.join(ROOT, "paper_1806_06698_amd", "csrc", "syev3_api.cpp")).read()
    old = "    if (o != g_seg_out && overlap(o[-1], ra)) return SYEV3_E_ALIAS;"
    assert src.count(old) == 1
    mut = tmp_path / "mutant"
    mut.mkdir()
    (mut / "syev3_api.cpp").write_text(src.replace(old, "    (void)o;"))
    exe = _build(tmp_path, str(mut), "api_segments_mutant")
    p = _run(exe, 100_000)
    assert p.returncode != 0 and "invalid segment call accepted" in p.stderr
