"""The graph compiler and the bundle reader under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only, CPU): tests/asan_driver.cpp is
built with hipcc, the sanitizers applied to the host side only, together with
the compiler's source; it compiles bundles of every algebra (with and without
outside-space records), reads them back with full validation and feeds the
reader corrupted and truncated copies.  Any sanitizer report or unexpected
status fails the test."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.slow
def test_compiler_and_reader_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "asan_driver")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-pthread"] + san + [
        "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "asan_driver.cpp"),
        os.path.join(ROOT, "paper_2609_14831_amd", "csrc", "builder.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=600, env=env)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("0 failures")
