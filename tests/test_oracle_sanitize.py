"""The oracle's C core under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): oracle/sanitize_check.c calls every entry point of
oracle/swr_oracle.c on small inputs (all potential kinds, every transmission
operator, interface and wall ends, optional outputs present and absent).  Any
out-of-bounds access, use after free, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "sanitize_check.c"), os.path.join(ROOT, "oracle", "swr_oracle.c")]


def test_oracle_core_is_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_check")
    build = subprocess.run([gcc, "-std=gnu99", "-g", "-O1", "-fno-omit-frame-pointer",
                            "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                            "-Wall", "-Wextra", "-o", exe, *SRC, "-lm"],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtimes not installed")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip() == "ok"
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
