"""The C ABI without Python: tests/c/solve_from_c.c, built with the host C
compiler against include/reg.h, libreg.so and the HIP runtime, registers the
32^3 smooth case (rho_R = rho_T shifted by two cells) and prints its report;
the mismatch must fall and the solve succeed."""
import os
import subprocess
import tempfile

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1608_03630_amd")


def test_solve_from_plain_c():
    assert os.path.exists(os.path.join(PKG, "libreg.so")), "build the library first"
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "solve_from_c")
        cmd = ["gcc", "-std=c11", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
               os.path.join(ROOT, "tests", "c", "solve_from_c.c"), "-o", exe, "-L" + PKG, "-lreg",
               "-L/opt/rocm/lib", "-lamdhip64", "-lm", "-Wl,-rpath," + PKG + ":/opt/rocm/lib"]
        subprocess.run(cmd, check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout.split()
    status, n_iter, matvecs = map(int, out[:3])
    final, first = map(float, out[3:5])
    print(f"  from C: status {status}, {n_iter} Newton steps, {matvecs} matvecs, mismatch {first:.4f} -> {final:.4f}",
          flush=True)
    assert status == 0 and n_iter >= 1 and matvecs >= 1 and final < first < 1.0
