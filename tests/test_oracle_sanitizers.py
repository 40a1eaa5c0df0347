"""The oracle's C part built with the address and undefined-behaviour
sanitizers (gcc -fsanitize=address,undefined) and driven through every C
entry point on 2D (p = 0..4) and 3D (p = 0..3) meshes: no out-of-bounds
access, no use after free, no undefined arithmetic."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_c_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    src = os.path.join(HERE, "sanitize", "oracle_driver.c")
    build = subprocess.run(["gcc", "-g", "-O1", "-std=c11", "-D_DEFAULT_SOURCE", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe, src, "-lm"],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    # verify_asan_link_order=0: the sanitizer runtime need not come first
    # among preloaded libraries of the environment
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr
    assert run.stdout.count("rc 0") == 9
