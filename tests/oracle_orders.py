"""Observed convergence orders of the oracle's time discretisation, shared
by the order pins in test_oracle_transport.py and by the mutation test that
runs them against deliberately broken copies of the oracle.

Run as a script it prints the orders as JSON for the oracle build named by
the ORACLE_LIB environment variable.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

TWO_PI = 2 * np.pi

# (n, nt) levels refined jointly in h and dt
JOINT_LEVELS = ((16, 4), (32, 8), (48, 12))


def inner(u, w):
    h3 = np.prod([TWO_PI / m for m in u.shape[-3:]])
    return h3 * float(np.sum(u * w))


def orders(errs, sizes):
    """Observed orders log(e_i / e_{i+1}) / log(s_{i+1} / s_i)."""
    return [float(np.log(errs[i] / errs[i + 1]) / np.log(sizes[i + 1] / sizes[i])) for i in range(len(errs) - 1)]


def time_orders(orc, shape=(32, 32, 32)):
    """g and H vt at a fixed v = v*/2 with nt = 4, 8, 16 against nt = 128 on
    the same grid: relative L2 errors and their observed orders in dt."""
    case = synth.smooth_case(shape)
    rhoR = orc.transport_forward(orc.params(shape, 4, 1e-2), case["v_true"], case["rhoT"])
    v = 0.5 * case["v_true"]
    vt = synth.smooth_random_field(shape, 38, kmax=2, ncomp=3)

    def run(nt):
        P = orc.params(shape, nt, 1e-2)
        g, _, _ = orc.gradient(P, case["rhoT"], rhoR, v)
        return g, orc.hessian_matvec(P, case["rhoT"], v, vt)

    g_ref, H_ref = run(128)
    eg, eh = [], []
    for nt in (4, 8, 16):
        g, H = run(nt)
        eg.append(np.sqrt(inner(g - g_ref, g - g_ref) / inner(g_ref, g_ref)))
        eh.append(np.sqrt(inner(H - H_ref, H - H_ref) / inner(H_ref, H_ref)))
    return {"g_err": eg, "g_order": orders(eg, (4, 8, 16)), "H_err": eh, "H_order": orders(eh, (4, 8, 16))}


def symmetry_orders(orc):
    """Relative symmetry defect |<Hu,w> - <u,Hw>| / |<Hu,w>| at v = v*/2 over
    JOINT_LEVELS, and the sign of <Hu,u>."""
    defects, positive = [], True
    for n, nt in JOINT_LEVELS:
        shape = (n, n, n)
        case = synth.smooth_case(shape)
        P = orc.params(shape, nt, 1e-2)
        v = 0.5 * case["v_true"]
        u = synth.smooth_random_field(shape, 39, kmax=2, ncomp=3)
        w = synth.smooth_random_field(shape, 40, kmax=2, ncomp=3)
        Hu = orc.hessian_matvec(P, case["rhoT"], v, u)
        Hw = orc.hessian_matvec(P, case["rhoT"], v, w)
        a, b = inner(Hu, w), inner(u, Hw)
        defects.append(abs(a - b) / abs(a))
        positive = positive and inner(Hu, u) > 0
    return {"defect": defects, "order": orders(defects, [n for n, _ in JOINT_LEVELS]), "positive": positive}


def newton_orders(orc):
    """At v = v* (inverse crime, lam = 0) central differences of g against
    the GN matvec over JOINT_LEVELS."""
    defects = []
    for n, nt in JOINT_LEVELS:
        shape = (n, n, n)
        case = synth.smooth_case(shape)
        P = orc.params(shape, nt, 1e-2)
        vs = case["v_true"]
        rhoR = orc.transport_forward(P, vs, case["rhoT"])
        vt = synth.smooth_random_field(shape, 41, kmax=2, ncomp=3)
        H = orc.hessian_matvec(P, case["rhoT"], vs, vt)
        eps = 1e-4
        gp, _, _ = orc.gradient(P, case["rhoT"], rhoR, vs + eps * vt)
        gm, _, _ = orc.gradient(P, case["rhoT"], rhoR, vs - eps * vt)
        fd = (gp - gm) / (2 * eps)
        defects.append(np.sqrt(inner(fd - H, fd - H) / inner(H, H)))
    return {"defect": defects, "order": orders(defects, [n for n, _ in JOINT_LEVELS])}


def full_newton_orders(orc):
    """At v = v*/2 (lam != 0) central differences of g against the full Newton
    matvec and against the Gauss-Newton matvec over JOINT_LEVELS, and the
    Newton matvec's symmetry defect."""
    dn, dg, sym = [], [], []
    for n, nt in JOINT_LEVELS:
        shape = (n, n, n)
        case = synth.smooth_case(shape)
        P = orc.params(shape, nt, 1e-2)
        rhoR = orc.transport_forward(P, case["v_true"], case["rhoT"])
        v = 0.5 * case["v_true"]
        vt = synth.smooth_random_field(shape, 41, kmax=2, ncomp=3)
        Hn = orc.newton_matvec(P, case["rhoT"], rhoR, v, vt)
        Hg = orc.hessian_matvec(P, case["rhoT"], v, vt)
        eps = 1e-4
        gp, _, _ = orc.gradient(P, case["rhoT"], rhoR, v + eps * vt)
        gm, _, _ = orc.gradient(P, case["rhoT"], rhoR, v - eps * vt)
        fd = (gp - gm) / (2 * eps)
        dn.append(np.sqrt(inner(fd - Hn, fd - Hn) / inner(fd, fd)))
        dg.append(np.sqrt(inner(fd - Hg, fd - Hg) / inner(fd, fd)))
        u = synth.smooth_random_field(shape, 39, kmax=2, ncomp=3)
        w = synth.smooth_random_field(shape, 40, kmax=2, ncomp=3)
        Hu = orc.newton_matvec(P, case["rhoT"], rhoR, v, u)
        Hw = orc.newton_matvec(P, case["rhoT"], rhoR, v, w)
        sym.append(abs(inner(Hu, w) - inner(u, Hw)) / abs(inner(Hu, w)))
    sizes = [n for n, _ in JOINT_LEVELS]
    return {"newton": dn, "newton_order": orders(dn, sizes), "gauss_newton": dg, "symmetry": sym,
            "symmetry_order": orders(sym, sizes)}


if __name__ == "__main__":
    import oracle

    oracle._load()
    out = {"time": time_orders(oracle), "symmetry": symmetry_orders(oracle), "newton": newton_orders(oracle)}
    if "--full-newton" in sys.argv:
        out["full_newton"] = full_newton_orders(oracle)
    print(json.dumps(out, default=float))
