"""Failure paths of the C ABI on the GPU, each forced by its inputs (no
kernel faults): non-finite data (REG_ENONFINITE), a PCG run ended by
negative curvature (against the oracle, which takes the same exit), and a
folded map caught by the determinant check (REG_ENONDIFFEO)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import rel_l2, say, to_dev, to_host, to_vel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


@pytest.mark.parametrize("prec", [1, 0])
def test_nan_image_reports_nonfinite(reg, prec):
    shape = (16, 16, 16)
    case = synth.smooth_case(shape)
    rhoR = case["rhoT"].copy()
    rhoR[3, 4, 5] = np.nan
    ctx = reg.Context(reg.reg_default_params(shape, prec=prec, nt=4))
    ctx.reg_set_images(to_dev(case["rhoT"], ctx), to_dev(rhoR, ctx))
    with pytest.raises(reg.RegError) as e:
        ctx.reg_gradient(to_vel(0.1 * case["v_true"], ctx))
    assert e.value.status == reg.REG_ENONFINITE
    v0 = to_vel(np.zeros((3,) + shape), ctx)
    v, rep = ctx.reg_solve(v0, raise_on_error=False)
    assert rep["status"] == reg.REG_ENONFINITE and rep["n_iter"] == 0


def test_negative_curvature_exit_matches_oracle(reg):
    """rho_R = -5 rho_T shifted by four cells, beta = 1e-3, started from
    twice the paper's velocity: with the full Hessian (the Gauss-Newton one
    is positive) the first PCG direction has negative curvature (about
    -0.59 <p,p>), so PCG stops at once and the step is -M g; one Newton
    step, in double."""
    hessian = 1
    shape, nt = (16, 16, 16), 4
    case = synth.smooth_case(shape)
    rhoT = case["rhoT"]
    rhoR = -5.0 * np.roll(rhoT, 4, axis=0)
    v0 = 2.0 * synth.smooth_velocity_paper(shape)
    P = oracle.params(shape, nt, 1e-3, max_newton=1, hessian=hessian)
    v_ref, rep_ref = oracle.solve(P, rhoT, rhoR, v0)
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=1, beta=1e-3, max_newton=1, hessian=hessian))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    v, rep = ctx.reg_solve(to_vel(v0, ctx))
    say(f"  hessian {hessian}: gpu neg-curv {rep['negative_curvature']} pcg {rep['pcg_iters']} J {rep['J']}; "
        f"oracle neg-curv {rep_ref['negative_curvature']} pcg {rep_ref['pcg_iters']} J {rep_ref['J']}")
    assert rep_ref["negative_curvature"] == 1 and rep_ref["pcg_iters"] == [1]
    assert rep["negative_curvature"] == rep_ref["negative_curvature"]
    assert rep["pcg_iters"] == rep_ref["pcg_iters"] and rep["status"] == rep_ref["status"] == 0
    assert rel_l2(to_host(v), v_ref) <= 1e-9


@pytest.mark.parametrize("prec", [1, 0])
def test_det_check(reg, prec):
    """det_check computes det grad y1 of the result (as reg_deformation
    does) and returns REG_ENONDIFFEO for a folded map: ten times the paper's
    velocity in one time step folds the grid (det min about -1.9e4 in the
    oracle)."""
    shape = (16, 16, 16)
    case = synth.smooth_case(shape)
    rhoR = oracle.transport_forward(oracle.params(shape, 4, 1e-2), case["v_true"], case["rhoT"])
    ctx = reg.Context(reg.reg_default_params(shape, prec=prec, nt=4, max_newton=2, det_check=1))
    ctx.reg_set_images(to_dev(case["rhoT"], ctx), to_dev(rhoR, ctx))
    v, rep = ctx.reg_solve()
    _, dmin, dmax = ctx.reg_deformation(v)
    assert rep["status"] == 0 and 0 < rep["det_min"] <= 1 <= rep["det_max"]
    assert rep["det_min"] == dmin and rep["det_max"] == dmax
    assert rep["fft3d"] > 0 and rep["fft_lines"] > 0
    fold = reg.Context(reg.reg_default_params(shape, prec=prec, nt=1, max_newton=0, det_check=1))
    fold.reg_set_images(to_dev(case["rhoT"], fold), to_dev(rhoR, fold))
    v0 = to_vel(10.0 * synth.smooth_velocity_paper(shape), fold)
    v, rep = fold.reg_solve(v0, raise_on_error=False)
    _, _, mn, _ = oracle.deformation(oracle.params(shape, 1, 1e-2), 10.0 * synth.smooth_velocity_paper(shape))
    say(f"  prec {prec}: det min {rep['det_min']:.4g} (oracle {mn:.4g})")
    assert rep["status"] == reg.REG_ENONDIFFEO and rep["det_min"] < 0
    assert abs(rep["det_min"] - mn) <= (1e-10 if prec else 1e-4) * abs(mn)
