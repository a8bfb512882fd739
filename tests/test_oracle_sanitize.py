"""The FP64 oracle under AddressSanitizer, UndefinedBehaviorSanitizer and LeakSanitizer:
oracle/oracle.c and a driver (tests/sanitize_oracle.c) built with gcc and run as a child
process, one thread and three threads, 2- to 5-way ragged shapes with and without a zero
factor column.  Any out-of-bounds access, use of freed memory, leak or undefined operation
ends the run with a report and a non-zero status."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_oracle")
    cmd = [gcc, "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe, os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(HERE, "sanitize_oracle.c"), "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr + b.stdout).lower():
        pytest.skip("sanitizer runtime not available: " + b.stderr[-200:])
    assert b.returncode == 0, b.stderr
    # verify_asan_link_order=0: the runtime need not come first among preloaded libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize driver ok" in r.stdout
    assert "runtime error" not in r.stderr
