"""recompute_grad_rho = 1: the workspace keeps one level of grad rho^n
instead of nt + 1, and the gradient, the Hessian matvec and the solve
recompute grad rho^n by line FFTs (section III-C1) wherever they need it.
Against the contexts that keep every level: the same gradient, matvec and
solve (the same derivative kernels on the same state history, the b sum in
the same order of additions) in both precisions, single and batched (with
the matvec graph replayed), and against the oracle; the workspace is 3 nt
fields smaller; a context created without the room cannot be switched
back."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import TOL, biharm_bound, rel_l2, rounded, say, to_dev, to_host, to_vel

pytestmark = pytest.mark.gpu

# shape, nt, isochoric
PROBLEMS = [((64, 64, 64), 4, 0), ((32, 48, 64), 3, 1), ((24, 36, 54), 4, 0)]
BETA = 1e-2


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


def _case(shape, nt, iso, i, prec):
    case = synth.blob_case(shape, seed=2500 + i)
    rhoT = rounded(case["rhoT"], prec)
    P = oracle.params(shape, nt, BETA, isochoric=bool(iso))
    rhoR = rounded(oracle.transport_forward(P, case["v_true"], rhoT), prec)
    v = rounded(0.3 * case["v_true"], prec)
    vt = rounded(synth.smooth_random_field(shape, 2600 + i, kmax=3, ncomp=3), prec)
    return P, rhoT, rhoR, v, vt


@pytest.mark.parametrize("prec", [1, 0])
def test_gradient_and_matvec_equal_the_kept_levels(reg, prec):
    tol = 1e-13 if prec else 1e-6
    for i, (shape, nt, iso) in enumerate(PROBLEMS):
        P, rhoT, rhoR, v, vt = _case(shape, nt, iso, i, prec)
        out = []
        for rec in (0, 1):
            p = reg.reg_default_params(shape, nt=nt, prec=prec, beta=BETA, isochoric=iso, recompute_grad_rho=rec)
            ctx = reg.Context(p)
            ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
            g, J, mis, gn = ctx.reg_gradient(to_vel(v, ctx))
            H = ctx.reg_hessian_matvec(to_vel(vt, ctx))
            out.append((to_host(g), J, to_host(H), reg.reg_workspace_size(p)))
            ctx.close()
        (g0, J0, H0, w0), (g1, J1, H1, w1) = out
        esz = 8 if prec else 4
        eg, eh = rel_l2(g1, g0), rel_l2(H1, H0)
        say(f"  {shape} nt {nt} iso {iso} prec {prec}: gradient {eg:.1e}, matvec {eh:.1e}, workspace "
            f"{w0 / 2**20:.0f} -> {w1 / 2**20:.0f} MiB")
        assert eg <= tol and eh <= tol and abs(J1 - J0) <= tol * J0
        assert w0 - w1 == 3 * nt * np.prod(shape) * esz
        # and the oracle, at the usual bars
        g_ref, J_ref, mis_ref = oracle.gradient(P, rhoT, rhoR, v)
        H_ref = oracle.hessian_matvec(P, rhoT, v, vt)
        htol = (1e-12 if prec else 1e-4) + biharm_bound(shape, 1, BETA * np.linalg.norm(vt), np.linalg.norm(H_ref))
        assert abs(J1 - J_ref) <= TOL[("scalar", prec)] * J_ref
        assert rel_l2(H1, H_ref) <= htol


def test_solve_matches_the_oracle(reg):
    """The 32^3 smooth case in double, as with every level kept: the oracle's
    PCG counts per Newton step and its velocity to 1e-9."""
    shape, nt = (32, 32, 32), 4
    case = synth.smooth_case(shape)
    P = oracle.params(shape, nt, 1e-2, max_newton=5)
    rhoR = oracle.transport_forward(P, case["v_true"], case["rhoT"])
    v_ref, rep_ref = oracle.solve(P, case["rhoT"], rhoR)
    ctx = reg.Context(reg.reg_default_params(shape, nt=nt, prec=1, max_newton=5, recompute_grad_rho=1))
    ctx.reg_set_images(to_dev(case["rhoT"], ctx), to_dev(rhoR, ctx))
    v, rep = ctx.reg_solve()
    say(f"  gpu pcg {rep['pcg_iters']} oracle pcg {rep_ref['pcg_iters']}, fft lines {rep['fft_lines']}")
    assert rep["pcg_iters"] == rep_ref["pcg_iters"] and rep["n_iter"] == rep_ref["n_iter"]
    assert rel_l2(to_host(v), v_ref) <= 1e-9


def test_batch_with_recomputation_matches_single(reg):
    """A batch whose problems recompute grad rho (the per-step gradients run
    between the batched launches, and inside the captured matvec graph)
    gives, bit for bit, the single contexts' gradients and matvecs."""
    prec = 0
    params = [reg.reg_default_params(s, nt=nt, prec=prec, beta=BETA, isochoric=iso, recompute_grad_rho=1)
              for s, nt, iso in PROBLEMS]
    data = [_case(s, nt, iso, i, prec) for i, (s, nt, iso) in enumerate(PROBLEMS)]
    b = reg.Batch(params)
    for i, (_, rhoT, rhoR, _, _) in enumerate(data):
        ctx = b.contexts[i]
        b.reg_set_images(i, to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    vs = [to_vel(d[3], ctx) for d, ctx in zip(data, b.contexts)]
    vts = [to_vel(d[4], ctx) for d, ctx in zip(data, b.contexts)]
    gb, Jb, _, _ = b.reg_batch_gradient(vs)
    Hb = []
    for call in range(3):  # eager, captured, replayed
        Hb = b.reg_batch_hessian_matvec(vts)
        torch.cuda.synchronize()
    for i, (p, (_, rhoT, rhoR, v, vt)) in enumerate(zip(params, data)):
        ctx = reg.Context(p)
        ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
        g, J, _, _ = ctx.reg_gradient(to_vel(v, ctx))
        H = ctx.reg_hessian_matvec(to_vel(vt, ctx))
        torch.cuda.synchronize()
        assert torch.equal(gb[i], g) and Jb[i] == J, f"gradient of problem {i}"
        assert torch.equal(Hb[i], H), f"matvec of problem {i}"
        ctx.close()
    say(f"  batch stats {b.reg_batch_stats()}")


def test_cannot_turn_the_cache_back_on(reg):
    shape = (32, 32, 32)
    ctx = reg.Context(reg.reg_default_params(shape, nt=4, recompute_grad_rho=1))
    with pytest.raises(reg.RegError) as e:
        ctx.reg_set_solver(reg.reg_default_params(shape, nt=4, recompute_grad_rho=0))
    assert e.value.status == reg.REG_EINVAL
    ctx2 = reg.Context(reg.reg_default_params(shape, nt=4))
    ctx2.reg_set_solver(reg.reg_default_params(shape, nt=4, recompute_grad_rho=1))  # room to spare: allowed
