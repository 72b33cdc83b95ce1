"""Pins of the oracle's Gauss-Newton-Krylov solver (section III-A of the
paper: Armijo-globalised Newton, inexact PCG with a gradient-dependent
tolerance, the inverse biharmonic preconditioner, beta continuation) and of
its failure paths. The paper prints no per-iteration values, so parity with
the paper itself is unpinned; these tests check what must hold for any
correct run plus the stored oracle regression fixture."""
import json
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
TWO_PI = 2 * np.pi


def inner(u, w):
    h3 = np.prod([TWO_PI / m for m in u.shape[-3:]])
    return h3 * float(np.sum(u * w))


@pytest.fixture(scope="module")
def smooth32(orc):
    shape = (32, 32, 32)
    c = synth.smooth_case(shape)
    P = orc.params(shape, 4, 1e-2, max_newton=5)
    rhoR = orc.transport_forward(P, c["v_true"], c["rhoT"])
    return shape, c["rhoT"], rhoR


def test_smooth_case_converges_monotonically(orc, smooth32):
    shape, rhoT, rhoR = smooth32
    P = orc.params(shape, 4, 1e-2, max_newton=5)
    J0, _ = orc.objective(P, rhoT, rhoR, np.zeros((3,) + shape))
    v, rep = orc.solve(P, rhoT, rhoR)
    assert rep["status"] == 0 and rep["stop_reason"] == 0
    J = [J0] + rep["J"]
    assert all(J[i + 1] < J[i] for i in range(len(J) - 1)), J
    assert rep["grel"][-1] <= 1e-2
    # the reported final values are those of the returned velocity
    g, Jv, mis = orc.gradient(P, rhoT, rhoR, v)
    assert abs(Jv - rep["final_J"]) <= 1e-12 * Jv
    assert abs(mis - rep["final_mismatch"]) <= 1e-12


def test_matches_stored_oracle_fixture(orc, smooth32):
    """Regression against the report written by tests/golden/make_golden.py."""
    shape, rhoT, rhoR = smooth32
    with open(os.path.join(HERE, "golden", "smooth32_solve.json")) as f:
        gold = json.load(f)
    P = orc.params(shape, 4, 1e-2, max_newton=5)
    _, rep = orc.solve(P, rhoT, rhoR)
    assert rep["pcg_iters"] == gold["pcg_iters"]
    assert np.allclose(rep["J"], gold["J"], rtol=1e-10, atol=0)
    assert np.allclose(rep["mismatch"], gold["mismatch"], rtol=1e-10, atol=0)


def test_mismatch_stop(orc, smooth32):
    shape, rhoT, rhoR = smooth32
    P = orc.params(shape, 4, 1e-2, max_newton=5, mismatch_tol=0.8)
    _, rep = orc.solve(P, rhoT, rhoR)
    assert rep["stop_reason"] == 1 and rep["n_iter"] >= 1
    assert rep["mismatch"][-1] <= 0.8 and all(m > 0.8 for m in rep["mismatch"][:-1])


def test_line_search_failure_keeps_velocity(orc, smooth32):
    """With no line-search trials allowed no step can be accepted: the solver
    reports the failure and leaves v at its input."""
    shape, rhoT, rhoR = smooth32
    P = orc.params(shape, 4, 1e-2, max_newton=5, max_ls=0)
    v0 = 0.01 * synth.smooth_velocity_paper(shape)
    v, rep = orc.solve(P, rhoT, rhoR, v0)
    assert rep["status"] == 6
    assert np.array_equal(v, v0)


def test_beta_continuation_levels(orc):
    shape = (16, 16, 16)
    c = synth.smooth_case(shape)
    P0 = orc.params(shape, 4, 1e-2)
    rhoR = orc.transport_forward(P0, c["v_true"], c["rhoT"])
    P = orc.params(shape, 4, 1e-1, beta_final=1e-3, beta_factor=0.1, max_newton=4)
    _, rep = orc.solve(P, c["rhoT"], rhoR)
    levels = sorted(set(rep["beta"]), reverse=True)
    assert np.allclose(levels, [1e-1, 1e-2, 1e-3][: len(levels)]) and len(levels) >= 2
    # mismatch improves as beta falls
    assert rep["mismatch"][-1] < rep["mismatch"][0]


def test_loose_intermediate_levels_and_absolute_reference(orc):
    """gtol_level stops each level above beta_final as soon as |g| <= gtol_level
    |g0| (and not before); the last level runs to gtol. gnorm_ref replaces
    |g0| by an absolute reference."""
    shape = (16, 16, 16)
    c = synth.smooth_case(shape)
    P0 = orc.params(shape, 4, 1e-2)
    rhoR = orc.transport_forward(P0, c["v_true"], c["rhoT"])
    P = orc.params(shape, 4, 1e-1, beta_final=1e-3, beta_factor=0.1, max_newton=10, gtol_level=0.3)
    _, rep = orc.solve(P, c["rhoT"], rhoR)
    betas, grel = np.array(rep["beta"]), np.array(rep["grel"])
    for b in sorted(set(rep["beta"]), reverse=True):
        g = grel[betas == b]
        tol = 1e-2 if np.isclose(b, 1e-3) else 0.3
        assert g[-1] <= tol and np.all(g[:-1] > tol), (b, g)
    assert np.isclose(min(rep["beta"]), 1e-3)
    # an absolute reference ten times |g(v=0)| is met at once: no Newton step
    g_zero = orc.gradient(orc.params(shape, 4, 1e-1), c["rhoT"], rhoR, np.zeros((3,) + shape))[0]
    g0 = np.sqrt(inner(g_zero, g_zero))
    Pr = orc.params(shape, 4, 1e-1, max_newton=10, gnorm_ref=10 * g0 / 1e-2)
    _, rep2 = orc.solve(Pr, c["rhoT"], rhoR)
    assert rep2["n_iter"] == 0 and rep2["stop_reason"] == 0


def test_isochoric_solve_stays_divergence_free(orc):
    shape = (16, 16, 16)
    b = synth.blob_case(shape)
    P = orc.params(shape, 4, 1e-3, isochoric=True, max_newton=3)
    rhoR = orc.transport_forward(P, b["v_true"], b["rhoT"])
    v, rep = orc.solve(P, b["rhoT"], rhoR)
    assert rep["status"] == 0 and rep["n_iter"] >= 1
    dv = orc.div(v)
    assert np.sqrt(inner(dv, dv)) <= 1e-12 * np.sqrt(inner(v, v))


def test_preconditioned_cg_reduces_the_residual(orc, smooth32):
    """One Newton system solved to a tight tolerance: the Hessian is SPD at
    v = 0, so PCG from s = 0 must bring ||H s + g|| below eta ||g||."""
    shape, rhoT, rhoR = smooth32
    P = orc.params(shape, 4, 1e-2)
    v0 = np.zeros((3,) + shape)
    g, _, _ = orc.gradient(P, rhoT, rhoR, v0)
    # plain PCG written out here against the oracle's operators
    s = np.zeros_like(g)
    r = -g
    z = orc.precond(r, 1e-2)
    p = z.copy()
    rz = inner(r, z)
    for _ in range(30):
        q = orc.hessian_matvec(P, rhoT, v0, p)
        a = rz / inner(p, q)
        s += a * p
        r -= a * q
        if np.sqrt(inner(r, r)) <= 1e-6 * np.sqrt(inner(g, g)):
            break
        z = orc.precond(r, 1e-2)
        rz1 = inner(r, z)
        p = z + rz1 / rz * p
        rz = rz1
    res = orc.hessian_matvec(P, rhoT, v0, s) + g
    assert np.sqrt(inner(res, res)) <= 1e-6 * np.sqrt(inner(g, g))


def test_paper_parameters_fixture():
    """The paper's stated run parameters (section IV-A3), stored with their
    citation, are what the solver defaults must encode."""
    with open(os.path.join(HERE, "golden", "paper_parameters.json")) as f:
        gold = json.load(f)
    assert gold["beta"] == 1e-2 and gold["nt"] == 4 and gold["gtol"] == 1e-2


def test_grid_continuation_reaches_the_single_grid_minimiser(orc):
    """Grid continuation (coarse solve, spectral prolongation, fine solve)
    solves the fine problem: with the same absolute gradient tolerance
    (gnorm_ref = |g(0)|) the result agrees with the single-grid solve to about
    that tolerance, and the gap closes as the tolerance tightens. The
    prolonged coarse solution starts the fine grid well below |g(0)| (a wrong
    prolongation scale or restriction would not), and the fine grid needs
    fewer Newton steps than a cold start."""
    shape = (32, 32, 32)
    c = synth.smooth_case(shape)
    P0 = orc.params(shape, 4, 1e-2)
    rhoT = c["rhoT"]
    rhoR = orc.transport_forward(P0, c["v_true"], rhoT)
    g_zero = orc.gradient(P0, rhoT, rhoR, np.zeros((3,) + shape))[0]
    g0 = np.sqrt(inner(g_zero, g_zero))
    gaps = []
    for gtol in (1e-3, 1e-4):
        P = orc.params(shape, 4, 1e-2, max_newton=20, gtol=gtol, gnorm_ref=g0)
        v1, r1 = orc.solve(P, rhoT, rhoR)
        v2, r2 = orc.solve_grid(P, rhoT, rhoR, 2)
        assert r1["status"] == 0 and r2["status"] == 0 and r2["stop_reason"] == 0
        coarse, fine = r2["levels"]
        assert coarse["n"] == (16, 16, 16) and fine["n"] == shape
        assert fine["n_iter"] < r1["n_iter"]
        gaps.append(np.sqrt(inner(v1 - v2, v1 - v2) / inner(v1, v1)))
    assert gaps[1] <= 1e-3 and gaps[1] < 0.5 * gaps[0], gaps
    # the fine grid starts from the prolonged coarse solution
    Pc = orc.coarse_params(P0, (16, 16, 16))
    vc, _ = orc.solve(Pc, orc.resample(rhoT, 16), orc.resample(rhoR, 16))
    gp = orc.gradient(P0, rhoT, rhoR, orc.resample(vc, 32))[0]
    assert np.sqrt(inner(gp, gp)) <= 0.5 * g0


def test_grid_continuation_resumes_beta_where_the_coarse_grid_ended(orc):
    """Each grid of the continuation resumes the beta continuation at the
    level the coarser grid ended on, and the report lists the grids coarsest
    first."""
    shape = (16, 16, 16)
    c = synth.smooth_case(shape)
    P0 = orc.params(shape, 4, 1e-2)
    rhoR = orc.transport_forward(P0, c["v_true"], c["rhoT"])
    P = orc.params(shape, 4, 1e-1, beta_final=1e-3, max_newton=4, gtol_level=0.3)
    v, rep = orc.solve_grid(P, c["rhoT"], rhoR, 2)
    coarse, fine = rep["levels"]
    assert coarse["n"] == (8, 8, 8) and np.isclose(coarse["final_beta"], 1e-3)
    assert all(np.isclose(b, 1e-3) for b in fine["beta"]) and np.isclose(rep["final_beta"], 1e-3)
    # the resumed level keeps the gradient reference of its start on the
    # coarse grid: relative gradients are reported against it
    assert np.isclose(fine["final_gref"], coarse["final_gref"], rtol=0, atol=0)


def test_grid_continuation_stops_where_one_grid_would(orc):
    """Three grids (8^3, 16^3, 32^3) with beta continuation 1e-1 -> 1e-2:
    every grid ends by the gradient test against its level's reference, and
    the finest grid ends at |g| <= gtol times the reference taken where the
    last level began, on a coarser grid."""
    shape = (32, 32, 32)
    c = synth.smooth_case(shape)
    rhoR = orc.transport_forward(orc.params(shape, 4, 1e-2), c["v_true"], c["rhoT"])
    P = orc.params(shape, 4, 1e-1, beta_final=1e-2, max_newton=6, gtol_level=0.3)
    v, rep = orc.solve_grid(P, c["rhoT"], rhoR, 3)
    assert [l["n"][0] for l in rep["levels"]] == [8, 16, 32]
    assert all(l["status"] == 0 and l["stop_reason"] == 0 for l in rep["levels"])
    g = orc.gradient(orc.params(shape, 4, 1e-2), c["rhoT"], rhoR, v)[0]
    assert np.sqrt(inner(g, g)) <= 1e-2 * rep["final_gref"] * (1 + 1e-9)


def test_negative_curvature_exit_takes_the_steepest_descent_step(orc):
    """With rho_R = -5 rho_T shifted by four cells, beta = 1e-3 and the start
    v0 = 2 v_paper, the first PCG direction p = -M g has <p, H p> < 0 for the
    full Hessian (eqs. (5a)-(5e); the Gauss-Newton part is positive): PCG
    stops at once (section III-A truncates at negative curvature) and the
    Newton step is the preconditioned steepest descent step, so the accepted
    iterate is v0 - alpha M g with the reported alpha."""
    hessian = 1
    shape, nt = (16, 16, 16), 4
    c = synth.smooth_case(shape)
    rhoT = c["rhoT"]
    rhoR = -5.0 * np.roll(rhoT, 4, axis=0)
    v0 = 2.0 * synth.smooth_velocity_paper(shape)
    P = orc.params(shape, nt, 1e-3, max_newton=1, hessian=hessian)
    g = orc.gradient(P, rhoT, rhoR, v0)[0]
    p = orc.precond(-g, 1e-3)
    Hp = orc.newton_matvec(P, rhoT, rhoR, v0, p) if hessian else orc.hessian_matvec(P, rhoT, v0, p)
    assert inner(p, Hp) < 0
    v, rep = orc.solve(P, rhoT, rhoR, v0)
    assert rep["negative_curvature"] == 1 and rep["pcg_iters"] == [1] and rep["n_iter"] == 1
    assert np.allclose(v, v0 + rep["alpha"][0] * p, rtol=0, atol=1e-12 * np.abs(v0).max())
