"""Mutation check of the oracle's pins: compile copies of oracle.c with one
plausible first-order mistake each, and show that the mathematics-based
order pins (not only the stored regression fixture) reject them.

Mutants (each a single textual change of oracle.c; the full Newton ones are
listed at NEWTON_MUTANTS):
  * trapezoid: uniform weights 1/(nt+1) in the time quadrature of b and b~
    (eqs. (4), (5e) read with the trapezoid rule);
  * inc_source: the corrector of the incremental state (eq. (5a) advanced
    with eq. (7)) takes the source at t^n instead of t^{n+1}.
The mutants are built with gcc into a temporary directory and run in child
processes, so the oracle loaded by the other tests is untouched.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "trapezoid": (
        "static double trap_w(int k, int nt) { return (k == 0 || k == nt) ? 0.5 / nt : 1.0 / nt; }",
        "static double trap_w(int k, int nt) { return 1.0 / (nt + 1); }",
    ),
    "inc_source": (
        "rt[p] = nu0[p] + 0.5 * dt * (f0[p] + src[(long)(k + 1) * N + p]);",
        "rt[p] = nu0[p] + 0.5 * dt * (f0[p] + src[(long)(k) * N + p]);",
    ),
}


# mutants of the full Newton matvec (eqs. (5c), (5e) with the lam terms):
# the source div(lam vt) taken at x instead of at the departure point, and
# the term int lam grad rho~ dt of b~ with its sign flipped
NEWTON_MUTANTS = {
    "newton_source_point": (
        "double f00 = nu0[p] * cX + sX[p];",
        "double f00 = nu0[p] * cX + sk[(long)k * N + p];",
    ),
    "newton_b_sign": (
        "bt[j * N + p] += w * lamg[(long)k * N + p] * gt[j * N + p];",
        "bt[j * N + p] -= w * lamg[(long)k * N + p] * gt[j * N + p];",
    ),
}


def _build(tmp_path, name):
    text = open(SRC).read()
    old, new = {**MUTANTS, **NEWTON_MUTANTS}[name]
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / f"{name}.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-std=c11", "-O3", "-march=x86-64-v2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", str(src), "-o", str(lib), "-lm"], check=True)
    return str(lib)


def _orders(lib, *flags):
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "oracle_orders.py"), *flags], env=env,
                       capture_output=True, text=True, timeout=600, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def _passes_pins(o):
    """The thresholds of the order pins in test_oracle_transport.py."""
    return (min(o["time"]["g_order"]) >= 1.6 and min(o["time"]["H_order"]) >= 1.6
            and min(o["symmetry"]["order"]) >= 2.0 and min(o["newton"]["order"]) >= 2.0)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_order_pins_reject_first_order_mutants(tmp_path, name):
    o = _orders(_build(tmp_path, name))
    assert not _passes_pins(o), (name, o)
    # each mutant drops the time order of g or of H vt to about one
    assert min(o["time"]["g_order"] + o["time"]["H_order"]) < 1.3, (name, o)


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(NEWTON_MUTANTS))
def test_full_newton_pin_rejects_mutants(tmp_path, name):
    o = _orders(_build(tmp_path, name), "--full-newton")["full_newton"]
    # the thresholds of test_full_newton_matvec_is_the_derivative_of_the_gradient
    assert not (min(o["newton_order"]) >= 2.0 and o["newton"][-1] <= 0.01), (name, o)
