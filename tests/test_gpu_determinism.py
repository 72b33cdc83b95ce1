"""Run-to-run determinism. No kernel of the library uses atomics or
order-dependent reductions: every sum (the FP64 inner products, the b
quadrature, the network's weight gradients) has a fixed tree. So the same
call on the same inputs gives the same bits, in a second call on the same
context, and in a fresh context created on a workspace filled with NaN bytes
(nothing reads workspace memory it has not written).
Checked for the gradient, the Hessian matvec, the forward transport and a
whole solve (velocity and report), in both precisions."""
import ctypes

import pytest
import torch

import oracle
import synth
from gpu_util import rounded, say, to_dev, to_vel

pytestmark = pytest.mark.gpu

REPORT_KEYS = ("status", "n_iter", "matvecs", "gradients", "objectives", "stop_reason", "J", "mismatch", "grel",
               "alpha", "beta", "pcg_iters", "ls_trials", "final_J", "final_mismatch", "final_grel", "interps",
               "fft3d", "fft_lines", "det_min", "det_max")


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


def _poisoned_context(reg, p):
    """A context created by reg_create on a workspace that holds NaN bytes
    (0xFF) everywhere; close it with _close_poisoned."""
    nbytes = reg.reg_workspace_size(p)
    ws = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    h = ctypes.c_void_p()
    reg._chk(reg.lib().reg_create(ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), nbytes, reg._stream_ptr(None),
                                  ctypes.byref(h)), what="reg_create")
    ctx = reg.Context(p, borrowed=h)
    ctx.poisoned_workspace = ws  # the context's memory: kept alive with it
    return ctx


def _close_poisoned(reg, ctx):
    torch.cuda.synchronize()
    reg.lib().reg_destroy(ctx.handle)
    ctx.handle = None


def _calls(ctx, rhoT, rhoR, v, vt):
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    g, J, mis, gn = ctx.reg_gradient(to_vel(v, ctx))
    H = ctx.reg_hessian_matvec(to_vel(vt, ctx))
    r1 = ctx.reg_transport_forward(to_vel(v, ctx), to_dev(rhoT, ctx))
    torch.cuda.synchronize()
    return [g.clone(), H.clone(), r1.clone()], (J, mis, gn)


@pytest.mark.parametrize("shape,nt,iso,prec", [((64, 64, 64), 4, 0, 0), ((24, 36, 54), 3, 1, 1)])
def test_repeat_and_fresh_context_give_the_same_bits(reg, shape, nt, iso, prec):
    case = synth.blob_case(shape, seed=3100)
    rhoT = rounded(case["rhoT"], prec)
    P = oracle.params(shape, nt, 1e-2, isochoric=bool(iso))
    rhoR = rounded(oracle.transport_forward(P, case["v_true"], rhoT), prec)
    v = 0.4 * case["v_true"]
    vt = synth.smooth_random_field(shape, 3101, kmax=3, ncomp=3)
    p = reg.reg_default_params(shape, nt=nt, prec=prec, beta=1e-2, isochoric=iso)
    ctx = reg.Context(p)
    a, sa = _calls(ctx, rhoT, rhoR, v, vt)
    b, sb = _calls(ctx, rhoT, rhoR, v, vt)
    ctx.close()
    ctx2 = _poisoned_context(reg, p)
    c, sc = _calls(ctx2, rhoT, rhoR, v, vt)
    _close_poisoned(reg, ctx2)
    for name, x, y, z in zip(("gradient", "matvec", "transport"), a, b, c):
        assert torch.equal(x, y), f"{name}: second call differs"
        assert torch.equal(x, z), f"{name}: fresh context differs"
        assert torch.isfinite(x).all(), name
    assert sa == sb == sc
    say(f"  {shape} prec {prec}: J {sa[0]:.6e} repeated bit for bit")


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_is_reproducible(reg, prec):
    shape, nt = (32, 32, 32), 4
    case = synth.smooth_case(shape)
    rhoT = rounded(case["rhoT"], prec)
    P = oracle.params(shape, nt, 1e-2)
    rhoR = rounded(oracle.transport_forward(P, case["v_true"], rhoT), prec)
    p = reg.reg_default_params(shape, nt=nt, prec=prec, beta=1e-2, beta_final=1e-3, max_newton=6)
    runs = []
    for fresh in (False, False, True):
        ctx = _poisoned_context(reg, p) if fresh else reg.Context(p)
        ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
        vel, rep = ctx.reg_solve()
        torch.cuda.synchronize()
        runs.append((vel.clone(), {k: rep[k] for k in REPORT_KEYS}))
        if fresh:
            _close_poisoned(reg, ctx)
        else:
            ctx.close()
    (v0, r0), (v1, r1), (v2, r2) = runs
    assert torch.equal(v0, v1) and torch.equal(v0, v2)
    assert r0 == r1 == r2
    say(f"  prec {prec}: {r0['n_iter']} Newton steps, {r0['matvecs']} matvecs, mismatch {r0['final_mismatch']:.4e}")


def test_network_forward_and_gradients_are_reproducible(reg):
    """The warm-start network at 32^3: the forward and the loss gradient
    (weight gradients reduced over fixed chunk slices, then a fixed tree)
    repeat bit for bit, also in a second network object."""
    import numpy as np
    from oracle import net as onet

    n = 32
    flat = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in onet.random_params(41)])
    T = torch.from_numpy(synth.smooth_random_field((n, n, n), 42, kmax=4).astype(np.float32)).cuda()
    R = torch.from_numpy(synth.smooth_random_field((n, n, n), 43, kmax=4).astype(np.float32)).cuda()
    tgt = torch.from_numpy(0.1 * synth.smooth_random_field((n, n, n), 44, kmax=3, ncomp=3).astype(np.float32)).cuda()
    out = []
    for _ in range(2):
        net = reg.Net(n)
        net.reg_net_set_params(torch.from_numpy(flat.astype(np.float32)).cuda())
        for _ in range(2):
            v = net.reg_net_forward(T, R).clone()
            loss, g = net.reg_net_loss_grad(T, R, tgt)
            torch.cuda.synchronize()
            out.append((v, loss, g.clone()))
    v0, l0, g0 = out[0]
    for v, l, g in out[1:]:
        assert torch.equal(v, v0) and l == l0 and torch.equal(g, g0)
    say(f"  network loss {l0:.6e} repeated bit for bit over 4 runs")
