"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/c/oracle_sanitized.c includes oracle/oracle.c, is built by gcc for the
host with both sanitizers (errors abort, leaks are reported) and OpenMP, and
drives every exported oracle routine on 8x12x16 and 10x12x6 grids, including
interpolation at displacements of several periods and three short solves.
A clean run prints "ok" and a finite checksum."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_clean_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitized")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               os.path.join(ROOT, "tests", "c", "oracle_sanitized.c"), "-o", exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    words = r.stdout.split()
    assert words[0] == "ok" and float(words[1]) == float(words[1])
