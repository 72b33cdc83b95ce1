"""Parity at the benchmark's shapes.

* The 256^3 phantom of the benchmark (nt = 16, single precision): one reduced
  gradient and one Gauss-Newton matvec against the oracle's, stored as
  scalars (tests/phantom256.py, tests/golden/phantom256_nt16.json) because the
  oracle needs minutes for them.
* Grids whose x1 and x2 lines have 256 points, so that the matvec's in-place
  256-point strided transforms run inside the gradient and Hessian assembly
  and inside the Krylov iteration (the first inverse pass reads the direction
  p in place there).
* The 128^3 isochoric blob problem: one FP64 gradient against the oracle, and
  the FP32 solve against the FP64 solve on the GPU."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import TOL, biharm_bound, rel_l2, rounded, say, to_dev, to_host, to_vel

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import phantom256 as ph  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


def test_phantom256_gradient_and_matvec_match_stored_oracle(reg):
    with open(os.path.join(HERE, "golden", "phantom256_nt16.json")) as f:
        gold = json.load(f)
    say("  [fullsize] building the 256^3 phantom inputs with the oracle")
    rhoT, rhoR, v, vt = ph.inputs(oracle)
    shape = rhoT.shape
    ctx = reg.Context(reg.reg_default_params(shape, nt=ph.NT, prec=0, beta=ph.BETA))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    g, J, mis, gn = ctx.reg_gradient(to_vel(v, ctx))
    g = to_host(g)
    H = to_host(ctx.reg_hessian_matvec(to_vel(vt, ctx)))
    # the bounds of the gradient and Hessian parity tests: transport error
    # amplified by |rho_T - rho_R| / |rho_1 - rho_R| and by the cancellation
    # kappa of g = beta lap^2 v + b, plus the |k|^4 amplification of
    # transform round-off in beta lap^2 v (double in both modes)
    amp = max(1.0, 1.0 / gold["mismatch"])
    kappa = (gold["reg_norm"] + gold["b_norm"]) / gold["g_l2"]
    tol = 1e-4 * amp * kappa + biharm_bound(shape, 1, ph.BETA * gold["v_l2"], gold["g_l2"])
    htol = 1e-4 + biharm_bound(shape, 1, ph.BETA * gold["vt_l2"], gold["H_l2"])
    h3 = np.prod([2 * np.pi / m for m in shape])
    say(f"  J {J:.8e} / {gold['J']:.8e}, mismatch {mis:.6e} / {gold['mismatch']:.6e}, "
        f"|g| {gn:.6e} / {gold['g_norm']:.6e}; bounds {tol:.1e} (g), {htol:.1e} (H)")
    assert abs(J - gold["J"]) <= TOL[("scalar", 0)] * gold["J"]
    assert abs(mis - gold["mismatch"]) <= TOL[("scalar", 0)] * gold["mismatch"]
    assert abs(gn - gold["g_norm"]) <= tol * gold["g_norm"]
    assert abs(ph.inner(H, vt) - gold["H_vt"]) <= htol * h3 * gold["H_l2"] * gold["vt_l2"]
    # A probe w of M independent standard normal values, drawn independently
    # of the computation, turns an error e into <e, w> ~ N(0, (h3 |e|)^2):
    # normalised by h3 |result| |w| / sqrt(M) it is the relative L2 error
    # times a standard normal, so 5 x the relative bound holds unless the
    # error exceeds that bound (a 5-sigma event otherwise).
    for k in range(ph.NPROBES):
        w = ph.probe(shape[0], k)
        unit = h3 * gold["probe_l2"][k] / np.sqrt(w.size)
        eg = abs(ph.inner(g, w) - gold["g_probe"][k]) / (unit * gold["g_l2"])
        eh = abs(ph.inner(H, w) - gold["H_probe"][k]) / (unit * gold["H_l2"])
        say(f"  probe {k}: gradient {eg:.2e}, Hessian {eh:.2e} (relative error times a unit normal)")
        assert eg <= 5 * tol and eh <= 5 * htol


def _smooth_inputs(shape, nt, prec):
    case = synth.smooth_case(shape)
    rhoT = rounded(case["rhoT"], prec)
    rhoR = rounded(oracle.transport_forward(oracle.params(shape, nt, 1e-2), case["v_true"], rhoT), prec)
    return rhoT, rhoR, case


@pytest.mark.parametrize("prec", [1, 0])
def test_gradient_and_hessian_with_256_point_x1_x2_lines(reg, prec):
    shape, nt, beta = (256, 256, 16), 4, 1e-2
    rhoT, rhoR, case = _smooth_inputs(shape, nt, prec)
    v = rounded(0.5 * case["v_true"], prec)
    vt = rounded(synth.smooth_random_field(shape, 121, kmax=6, ncomp=3), prec)
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=prec, beta=beta))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    g, J, mis, _ = ctx.reg_gradient(to_vel(v, ctx))
    g = to_host(g)
    H = to_host(ctx.reg_hessian_matvec(to_vel(vt, ctx)))
    P = oracle.params(shape, nt, beta)
    g_ref, J_ref, mis_ref = oracle.gradient(P, rhoT, rhoR, v)
    H_ref = oracle.hessian_matvec(P, rhoT, v, vt)
    reg_part = oracle.biharm(v, beta)
    kappa = (np.linalg.norm(reg_part) + np.linalg.norm(g_ref - reg_part)) / np.linalg.norm(g_ref)
    base = 1e-12 if prec else 1e-4
    tol = base * max(1.0, 1.0 / mis_ref) * kappa + biharm_bound(shape, 1, beta * np.linalg.norm(v),
                                                                 np.linalg.norm(g_ref))
    htol = base + biharm_bound(shape, 1, beta * np.linalg.norm(vt), np.linalg.norm(H_ref))
    say(f"  prec {prec}: gradient {rel_l2(g, g_ref):.2e} (bound {tol:.1e}), Hessian {rel_l2(H, H_ref):.2e} "
        f"(bound {htol:.1e})")
    assert rel_l2(g, g_ref) <= tol and rel_l2(H, H_ref) <= htol
    assert abs(J - J_ref) <= TOL[("scalar", prec)] * J_ref


@pytest.mark.parametrize("prec", [1, 0])
def test_solve_with_256_point_x1_lines_matches_oracle(reg, prec):
    """Every Krylov iteration's first inverse pass reads p in place through
    the 256-point strided transform when n1 = 256."""
    shape, nt = (256, 16, 64), 4
    rhoT, rhoR, _ = _smooth_inputs(shape, nt, prec)
    P = oracle.params(shape, nt, 1e-2, max_newton=5)
    v_ref, rep_ref = oracle.solve(P, rhoT, rhoR)
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=prec, max_newton=5))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    v, rep = ctx.reg_solve()
    say(f"  prec {prec}: gpu pcg {rep['pcg_iters']} mismatch {rep['final_mismatch']:.6f}; oracle pcg "
        f"{rep_ref['pcg_iters']} mismatch {rep_ref['final_mismatch']:.6f}; v rel-L2 {rel_l2(to_host(v), v_ref):.2e}")
    if prec:
        assert rep["pcg_iters"] == rep_ref["pcg_iters"]
        assert rel_l2(to_host(v), v_ref) <= 1e-9
    else:
        assert abs(rep["n_iter"] - rep_ref["n_iter"]) <= 1
        assert abs(rep["final_mismatch"] - rep_ref["final_mismatch"]) <= 0.01 * rep_ref["final_mismatch"]


def _blob128():
    shape, nt = (128, 128, 128), 8
    case = synth.blob_case(shape, seed=1002)
    P = oracle.params(shape, nt, 1e-3, isochoric=True)
    rhoT = rounded(case["rhoT"], 0)
    rhoR = rounded(oracle.transport_forward(P, case["v_true"], rhoT), 0)
    return shape, nt, P, rhoT, rhoR, case


def test_blob128_fp64_gradient_matches_oracle(reg):
    shape, nt, P, rhoT, rhoR, case = _blob128()
    v = 0.5 * case["v_true"]
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=1, beta=1e-3, isochoric=1))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    g, J, mis, _ = ctx.reg_gradient(to_vel(v, ctx))
    g_ref, J_ref, mis_ref = oracle.gradient(P, rhoT, rhoR, v)
    err = rel_l2(to_host(g), g_ref)
    tol = 1e-12 * max(1.0, 1.0 / mis_ref) + biharm_bound(shape, 1, 1e-3 * np.linalg.norm(v), np.linalg.norm(g_ref))
    say(f"  128^3 FP64 gradient rel-L2 {err:.2e} (bound {tol:.1e}), J {J:.12e} / {J_ref:.12e}")
    assert err <= tol and abs(J - J_ref) <= 1e-12 * J_ref and abs(mis - mis_ref) <= 1e-12 * mis_ref


def test_blob128_fp32_solve_tracks_fp64_solve(reg):
    """The 128^3 isochoric problem solved with FP32 fields and with FP64
    fields on the GPU (FP64 reductions and velocity in both): Newton steps
    within one, final mismatch within 1%; the velocity and final-state
    differences are reported."""
    shape, nt, P, rhoT, rhoR, case = _blob128()
    out = {}
    for prec in (1, 0):
        ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=prec, beta=1e-3, isochoric=1, max_newton=20))
        ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
        v, rep = ctx.reg_solve()
        rho1 = to_host(ctx.reg_transport_forward(v, to_dev(rhoT, ctx)))
        out[prec] = (to_host(v), rho1, rep)
        say(f"  prec {prec}: {rep['n_iter']} GN steps, {rep['matvecs']} matvecs, mismatch "
            f"{rep['final_mismatch']:.6f}, {rep['seconds_total']:.3f} s")
        del ctx
        torch.cuda.empty_cache()
    (v64, r64, rep64), (v32, r32, rep32) = out[1], out[0]
    say(f"  FP32 vs FP64: v rel-L2 {rel_l2(v32, v64):.2e}, rho1 rel-L2 {rel_l2(r32, r64):.2e}, mismatch "
        f"{rep32['final_mismatch']:.6f} vs {rep64['final_mismatch']:.6f}")
    assert abs(rep32["n_iter"] - rep64["n_iter"]) <= 1
    assert abs(rep32["final_mismatch"] - rep64["final_mismatch"]) <= 0.01 * rep64["final_mismatch"]
