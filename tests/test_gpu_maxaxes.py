"""The longest axes a context accepts (1024 points, and 512 and 1000 =
2^3 5^3) against the oracle. They take the LDS line transforms with a
single line per workgroup (two in single precision), the padded x3 tiles
and, at x3 = 1024, the canonical gather tiles of a long line. Each shape is
checked for the spectral operators, interpolation, the state and adjoint
transports, and one gradient and Hessian matvec, in both precisions, with the
parity tests' bounds."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (TOL, biharm_bound, biharm_fp32_bound, deriv_bound, rel_l2, rounded, say, to_dev, to_host,
                      to_vel)

pytestmark = pytest.mark.gpu

# x1 = 1024 (strided line transforms), x3 = 1024 (x3 tiles, canonical gathers),
# x1 = 1000 = 2^3 5^3 and x2 = 512, each with a short radix-5 x3 axis
SHAPES = [(1024, 8, 16), (8, 16, 1024), (1000, 8, 10), (16, 512, 10)]
SMALL = [(1024, 8, 16), (8, 16, 1024)]


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


def _lowpass(x, shape, kcut=8):
    """The part of x (..., n1, n2, n3) with |k_j| <= kcut on every axis."""
    X = np.fft.fftn(np.asarray(x, dtype=np.float64), axes=(-3, -2, -1))
    keep = np.ones(shape, dtype=bool)
    for j, n in enumerate(shape):
        k = np.abs(np.fft.fftfreq(n, 1.0 / n))
        sl = [None, None, None]
        sl[j] = slice(None)
        keep = keep & (k <= kcut)[tuple(sl)]
    return np.real(np.fft.ifftn(X * keep, axes=(-3, -2, -1)))


def _ctx(reg, shape, prec, nt=2, **kw):
    say(f"  [ctx] shape={shape} prec={prec} nt={nt} {kw}")
    return reg.Context(reg.reg_default_params(shape, nt=nt, prec=prec, **kw))


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("shape", SMALL)
def test_spectral_operators(reg, prec, shape):
    from paper_1608_03630_amd import reg as R

    ctx = _ctx(reg, shape, prec)
    u = rounded(synth.smooth_random_field(shape, 701, kmax=6), prec)
    ud = to_dev(u, ctx)
    for j in range(3):
        out = to_host(ctx.reg_deriv(j, ud))
        ref = oracle.deriv(u, j)
        tol = deriv_bound(shape, prec, {j: u}, ref)
        say(f"  d{j} rel-L2 {rel_l2(out, ref):.2e} (bound {tol:.2e})")
        assert rel_l2(out, ref) <= tol, j
    v = rounded(synth.smooth_random_field(shape, 702, kmax=6, ncomp=3), prec)
    vd = to_dev(v, ctx)
    d = to_host(ctx.reg_div(vd))
    ref = oracle.div(v)
    assert rel_l2(d, ref) <= deriv_bound(shape, prec, {0: v[0], 1: v[1], 2: v[2]}, ref)
    out = to_host(ctx.reg_spectral(R.SPEC_BIHARM, 0.01, vd))
    ref = oracle.biharm(v, 0.01)
    if prec:
        tol = max(TOL[("spectral", 1)], biharm_bound(shape, 1, np.linalg.norm(v), np.linalg.norm(ref / 0.01)))
    else:
        tol = biharm_fp32_bound(shape, v, ref / 0.01)
    say(f"  biharm rel-L2 {rel_l2(out, ref):.2e} (bound {tol:.2e})")
    assert rel_l2(out, ref) <= tol
    if tol > 1e-2:
        # In single precision on a 1024-point axis the transform's round-off
        # times |k|^4 (up to 512^4) outweighs lap^2 of a smooth field, so the
        # whole-band bound says little (the solver applies lap^2 in double).
        # The modes the field holds must still come out right: compare the
        # parts with |k_j| <= 8 on every axis.
        lo, lr = _lowpass(out, shape), _lowpass(ref, shape)
        say(f"  biharm |k| <= 8 rel-L2 {rel_l2(lo, lr):.2e}")
        assert rel_l2(lo, lr) <= 1e-5
    out = to_host(ctx.reg_spectral(R.SPEC_GAUSS, 0.3, vd))
    assert rel_l2(out, oracle.gauss(v, 0.3)) <= TOL[("spectral", prec)]
    out = to_host(ctx.reg_spectral(R.SPEC_LERAY, 0.0, vd))
    assert rel_l2(out, oracle.leray(v)) <= TOL[("spectral", prec)]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("shape", SMALL)
def test_interp_and_transport(reg, prec, shape):
    ctx = _ctx(reg, shape, prec, nt=3)
    f = rounded(synth.smooth_random_field(shape, 703, kmax=5), prec)
    D = rounded(synth.displacement(shape, 704, max_cells=2.5), prec)
    out = to_host(ctx.reg_interp(to_dev(f, ctx), to_dev(D, ctx)))
    e = rel_l2(out, oracle.interp(f, D))
    say(f"  interp rel-L2 {e:.2e}")
    assert e <= TOL[("interp", prec)]
    v = rounded(0.8 * synth.smooth_velocity_paper(shape), prec)
    P = oracle.params(shape, 3, 1e-2)
    r1 = to_host(ctx.reg_transport_forward(to_vel(v, ctx), to_dev(f, ctx)))
    assert rel_l2(r1, oracle.transport_forward(P, v, f)) <= TOL[("transport", prec)]
    l0 = to_host(ctx.reg_transport_adjoint(to_vel(v, ctx), to_dev(f, ctx)))
    assert rel_l2(l0, oracle.transport_adjoint(P, v, f)) <= TOL[("transport", prec)]


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("shape", SHAPES)
def test_gradient_and_matvec(reg, prec, shape):
    nt, beta = 2, 1e-2
    case = synth.smooth_case(shape)
    rhoT = rounded(case["rhoT"], prec)
    P = oracle.params(shape, nt, beta)
    rhoR = rounded(oracle.transport_forward(P, case["v_true"], rhoT), prec)
    v = rounded(0.5 * synth.smooth_velocity_paper(shape), prec)
    ctx = _ctx(reg, shape, prec, nt=nt, beta=beta)
    ctx.reg_set_images(to_dev(rhoT, ctx), to_dev(rhoR, ctx))
    g, J, mis, gn = ctx.reg_gradient(to_vel(v, ctx))
    g = to_host(g)
    g_ref, J_ref, mis_ref = oracle.gradient(P, rhoT, rhoR, v)
    # the gradient bar of the parity tests: transport error carried by the
    # residual (amp), cancellation in beta lap^2 v + P b (kappa), and
    # transform round-off amplified by |k|^4
    amp = max(1.0, 1.0 / max(mis_ref, 1e-300))
    reg_part = oracle.biharm(v, beta)
    kappa = (np.linalg.norm(reg_part) + np.linalg.norm(g_ref - reg_part)) / np.linalg.norm(g_ref)
    tol = (1e-12 if prec else 1e-4) * amp * kappa + biharm_bound(shape, 1, beta * np.linalg.norm(v),
                                                                  np.linalg.norm(g_ref))
    say(f"  gradient rel-L2 {rel_l2(g, g_ref):.2e} (bound {tol:.2e})")
    assert rel_l2(g, g_ref) <= tol
    assert abs(J - J_ref) <= TOL[("scalar", prec)] * abs(J_ref)
    vt = rounded(synth.smooth_random_field(shape, 705, kmax=3, ncomp=3), prec)
    H = to_host(ctx.reg_hessian_matvec(to_vel(vt, ctx)))
    H_ref = oracle.hessian_matvec(P, rhoT, v, vt)
    htol = (1e-12 if prec else 1e-4) + biharm_bound(shape, 1, beta * np.linalg.norm(vt), np.linalg.norm(H_ref))
    say(f"  Hessian rel-L2 {rel_l2(H, H_ref):.2e} (bound {htol:.2e})")
    assert rel_l2(H, H_ref) <= htol
