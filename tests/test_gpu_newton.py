"""GPU parity of the full Newton Hessian (reg_params.hessian = 1: eqs.
(5a)-(5e) with the source div(lam vt) in the incremental adjoint and
int lam grad rho~ dt in b~) against the oracle's newton_matvec, and of the
full Newton solve against the oracle's; Newton and Gauss-Newton iteration
counts side by side."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import biharm_bound, rel_l2, rounded, say, to_dev, to_host, to_vel

pytestmark = pytest.mark.gpu

RAGGED = (24, 36, 54)


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("iso", [False, True])
def test_newton_matvec_matches_oracle(reg, prec, iso):
    shape, nt, beta = RAGGED, 4, 1e-2
    case = synth.blob_case(shape, seed=1002) if iso else synth.smooth_case(shape)
    rhoT = rounded(case["rhoT"], prec)
    P = oracle.params(shape, nt, beta, isochoric=iso, hessian=1)
    rhoR = rounded(oracle.transport_forward(P, case["v_true"], rhoT), prec)
    v = rounded(0.5 * case["v_true"] if iso else 0.5 * synth.smooth_velocity_paper(shape), prec)
    vt = rounded(synth.smooth_random_field(shape, 130, kmax=3, ncomp=3), prec)
    if iso:
        vt = rounded(oracle.leray(vt), prec)
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=prec, beta=beta, isochoric=int(iso), hessian=1))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    ctx.reg_gradient(to_vel(v, ctx))
    H = to_host(ctx.reg_hessian_matvec(to_vel(vt, ctx)))
    H_ref = oracle.newton_matvec(P, rhoT, rhoR, v, vt)
    H_gn = oracle.hessian_matvec(P, rhoT, v, vt)
    tol = (1e-12 if prec else 1e-4) + biharm_bound(shape, 1, beta * np.linalg.norm(vt), np.linalg.norm(H_ref))
    err = rel_l2(H, H_ref)
    say(f"  prec {prec} iso {iso}: Newton matvec rel-L2 {err:.2e} (bound {tol:.1e}); "
        f"Newton vs Gauss-Newton {rel_l2(H_gn, H_ref):.2e}")
    assert err <= tol
    # the lam terms are not negligible here, so the test separates the two
    assert rel_l2(H_gn, H_ref) > 100 * tol


def test_newton_solve_fp64_matches_oracle(reg):
    """32^3 smooth case with the full Newton Hessian in double: the same PCG
    counts per Newton step and velocity to 1e-9; the Gauss-Newton solve of
    the same problem is reported beside it."""
    shape, nt = (32, 32, 32), 4
    case = synth.smooth_case(shape)
    rhoR = oracle.transport_forward(oracle.params(shape, nt, 1e-2), case["v_true"], case["rhoT"])
    out = {}
    for hessian in (1, 0):
        P = oracle.params(shape, nt, 1e-2, max_newton=8, gtol=1e-3, hessian=hessian)
        v_ref, rep_ref = oracle.solve(P, case["rhoT"], rhoR)
        ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=1, max_newton=8, gtol=1e-3, hessian=hessian))
        ctx.reg_set_images(to_dev(case["rhoT"], ctx), to_dev(rhoR, ctx))
        v, rep = ctx.reg_solve()
        say(f"  hessian={hessian}: gpu {rep['n_iter']} steps pcg {rep['pcg_iters']} grel {rep['final_grel']:.2e}; "
            f"oracle pcg {rep_ref['pcg_iters']}")
        assert rep["status"] == 0 and rep["pcg_iters"] == rep_ref["pcg_iters"]
        assert rel_l2(to_host(v), v_ref) <= 1e-9
        out[hessian] = rep
    say(f"  Newton {out[1]['n_iter']} steps / {out[1]['matvecs']} matvecs, Gauss-Newton {out[0]['n_iter']} steps / "
        f"{out[0]['matvecs']} matvecs to |g| <= 1e-3 |g0|")


def test_newton_needs_its_workspace(reg):
    ctx = reg.Context(reg.reg_default_params((16, 16, 16)))
    with pytest.raises(reg.RegError) as e:
        ctx.reg_set_solver(reg.reg_default_params((16, 16, 16), hessian=1))
    assert e.value.status == reg.REG_EINVAL
    ctx2 = reg.Context(reg.reg_default_params((16, 16, 16), hessian=1))
    ctx2.reg_set_solver(reg.reg_default_params((16, 16, 16), hessian=0))
