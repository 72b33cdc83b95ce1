"""Writes the stored oracle regression fixtures of this folder.

Calls only ``oracle`` (and the seeded input generators); run from the repo
root with ``python tests/golden/make_golden.py``."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def smooth32():
    shape = (32, 32, 32)
    c = synth.smooth_case(shape)
    P = oracle.params(shape, 4, 1e-2, max_newton=5)
    rhoR = oracle.transport_forward(P, c["v_true"], c["rhoT"])
    _, rep = oracle.solve(P, c["rhoT"], rhoR)
    keep = {k: rep[k] for k in ("n_iter", "matvecs", "J", "mismatch", "grel", "alpha", "pcg_iters", "ls_trials")}
    keep["workload"] = ("32^3 smooth case: rho_T = (sin^2 x1 + sin^2 x2 + sin^2 x3)/3, divergence-free "
                        "v* = (sin x3 cos x2 sin x2, sin x1 cos x3 sin x3, sin x2 cos x1 sin x1), "
                        "rho_R = oracle state solve, nt=4, beta=1e-2, gtol=1e-2, max 5 GN steps")
    with open(os.path.join(HERE, "smooth32_solve.json"), "w") as f:
        json.dump(keep, f, indent=1)


if __name__ == "__main__":
    smooth32()
