"""GPU parity of the grid-continued solve (reg_params.grid_levels) against the
oracle's solve_grid: images restricted by spectral truncation, each coarse
grid solved with the beta continuation, its velocity prolonged by spectral
zero-padding, the next grid resuming the continuation where the coarser one
ended. In double the per-grid Newton steps and matvecs equal the oracle's and
the velocity agrees to 1e-9; in single precision the outer steps stay within
one of the FP64 oracle and the final mismatch within 1%."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import rel_l2, rounded, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


def _smooth(shape, nt, prec):
    case = synth.smooth_case(shape)
    rhoT = rounded(case["rhoT"], prec)
    rhoR = rounded(oracle.transport_forward(oracle.params(shape, nt, 1e-2), case["v_true"], rhoT), prec)
    return rhoT, rhoR


def _levels_match(rep, rep_ref):
    got = [(tuple(l["n"]), l["n_iter"], l["matvecs"]) for l in rep["levels"]]
    want = [(tuple(l["n"]), l["n_iter"], l["matvecs"]) for l in rep_ref["levels"]]
    say(f"  gpu levels {got}\n  oracle levels {want}")
    return got == want


# The velocity bar follows the oracle's own sensitivity: a 1e-15 relative
# perturbation of rho_R moves its two-grid solution by about 1e-11 and its
# three-grid solution (8^3 coarsest, with beta continuation) by 1e-9 to 4e-9,
# and summation order differs from the oracle's by more than one such rounding.
@pytest.mark.parametrize("levels,kw,vtol", [
    (2, dict(beta=1e-2, max_newton=5), 1e-9),
    (3, dict(beta=1e-1, beta_final=1e-2, max_newton=6, gtol_level=0.3), 1e-7),
])
def test_grid_continuation_fp64_matches_oracle(reg, levels, kw, vtol):
    shape, nt = (32, 32, 32), 4
    rhoT, rhoR = _smooth(shape, nt, 1)
    P = oracle.params(shape, nt, kw["beta"], **{k: v for k, v in kw.items() if k != "beta"})
    v_ref, rep_ref = oracle.solve_grid(P, rhoT, rhoR, levels)
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=1, grid_levels=levels, **kw))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    log = []
    ctx.reg_set_log(log.append)
    v, rep = ctx.reg_solve()
    assert rep["status"] == 0 and len(rep["levels"]) == levels
    # every grid logs its accepted steps, coarsest first
    assert [sum(1 for e in log if e["n"] == list(l["n"])) for l in rep["levels"]] == \
        [l["n_iter"] for l in rep["levels"]]
    assert _levels_match(rep, rep_ref)
    assert rep["pcg_iters"] == rep_ref["pcg_iters"] and rep["beta"] == rep_ref["beta"]
    assert rel_l2(to_host(v), v_ref) <= vtol
    assert abs(rep["final_mismatch"] - rep_ref["final_mismatch"]) <= 1e-10
    for l, lr in zip(rep["levels"], rep_ref["levels"]):
        assert abs(l["final_mismatch"] - lr["final_mismatch"]) <= 1e-10
        assert np.isclose(l["final_beta"], lr["final_beta"], rtol=1e-12)


def test_grid_continuation_fp32_blob_tracks_oracle(reg):
    """Isochoric blob pair on 64^3 in single precision with a 32^3 coarse grid."""
    shape, nt = (64, 64, 64), 8
    case = synth.blob_case(shape, seed=1002)
    P = oracle.params(shape, nt, 1e-3, isochoric=True, max_newton=10, mismatch_tol=0.0)
    rhoT = rounded(case["rhoT"], 0)
    rhoR = rounded(oracle.transport_forward(P, case["v_true"], rhoT), 0)
    v_ref, rep_ref = oracle.solve_grid(P, rhoT, rhoR, 2)
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=0, beta=1e-3, isochoric=1, max_newton=10,
                                             grid_levels=2))
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    v, rep = ctx.reg_solve()
    got = [(l["n_iter"], round(l["final_mismatch"], 5)) for l in rep["levels"]]
    want = [(l["n_iter"], round(l["final_mismatch"], 5)) for l in rep_ref["levels"]]
    say(f"  gpu {got} oracle {want}; v rel-L2 {rel_l2(to_host(v), v_ref):.2e}")
    for l, lr in zip(rep["levels"], rep_ref["levels"]):
        assert abs(l["n_iter"] - lr["n_iter"]) <= 1
        assert abs(l["final_mismatch"] - lr["final_mismatch"]) <= 0.01 * lr["final_mismatch"]


def test_grid_levels_validation(reg):
    """A grid whose coarse levels are not valid sizes is refused, and
    reg_set_solver may lower grid_levels but not raise it past the workspace."""
    with pytest.raises(reg.RegError):
        reg.Context(reg.reg_default_params((24, 24, 24), grid_levels=3))  # 6 < 8
    ctx = reg.Context(reg.reg_default_params((32, 32, 32), grid_levels=2))
    ctx.reg_set_solver(reg.reg_default_params((32, 32, 32), grid_levels=1))
    with pytest.raises(reg.RegError) as e:
        ctx.reg_set_solver(reg.reg_default_params((32, 32, 32), grid_levels=3))
    assert e.value.status == reg.REG_EINVAL
