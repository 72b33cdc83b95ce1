"""Writes the stored oracle regression fixtures of this folder.

Calls only ``oracle`` (and the seeded input generators); run from the repo
root with ``python tests/golden/make_golden.py [smooth32] [phantom256]``
(phantom256 takes several minutes on the host)."""
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


def phantom256():
    """Scalars of the oracle's gradient and Gauss-Newton matvec on the 256^3
    benchmark phantom (nt = 16, beta = 1e-3, v = v_true / 2): several minutes
    on the host, so stored (see tests/phantom256.py)."""
    sys.path.insert(0, os.path.dirname(HERE))
    import numpy as np

    import phantom256 as ph

    rhoT, rhoR, v, vt = ph.inputs(oracle)
    shape = rhoT.shape
    P = oracle.params(shape, ph.NT, ph.BETA)
    g, J, mis = oracle.gradient(P, rhoT, rhoR, v)
    reg_part = oracle.biharm(v, ph.BETA)
    H = oracle.hessian_matvec(P, rhoT, v, vt)
    out = {
        "workload": ("256^3 ellipsoid phantom (seed 1003) smoothed by the oracle's Gaussian (sigma = 2 h), "
                     "rho_R = oracle state solve under v_true with nt = 16, v = v_true / 2, vt = seeded smooth "
                     "field (kmax 8, seed 120), beta = 1e-3, all inputs rounded to float32"),
        "J": J, "mismatch": mis,
        "g_norm": np.sqrt(ph.inner(g, g)), "reg_norm": float(np.linalg.norm(reg_part)),
        "b_norm": float(np.linalg.norm(g - reg_part)), "g_l2": float(np.linalg.norm(g)),
        "v_l2": float(np.linalg.norm(v)), "vt_l2": float(np.linalg.norm(vt)),
        "H_l2": float(np.linalg.norm(H)), "H_vt": ph.inner(H, vt),
        "g_probe": [], "H_probe": [], "probe_l2": [],
    }
    for k in range(ph.NPROBES):
        w = ph.probe(shape[0], k)
        out["g_probe"].append(ph.inner(g, w))
        out["H_probe"].append(ph.inner(H, w))
        out["probe_l2"].append(float(np.linalg.norm(w)))
    with open(os.path.join(HERE, "phantom256_nt16.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    which = sys.argv[1:] or ["smooth32"]
    if "smooth32" in which:
        smooth32()
    if "phantom256" in which:
        phantom256()
