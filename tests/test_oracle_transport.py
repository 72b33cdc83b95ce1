"""Pins of the oracle's semi-Lagrangian transport solves (eqs. (2b), (3),
(5a), (5c) advanced with eqs. (6)-(7)), the reduced gradient (eq. (4)), the
Gauss-Newton Hessian (eqs. (5a)-(5e) without the adjoint terms, section II-B)
and the deformation map (eq. (1)): exact special cases, closed forms at
v = 0, conservation and adjoint identities, and convergence orders."""
import numpy as np
import pytest

import synth
from oracle_orders import JOINT_LEVELS, full_newton_orders, newton_orders, orders, symmetry_orders, time_orders

TWO_PI = 2 * np.pi


def inner(u, w):
    h3 = np.prod([TWO_PI / m for m in u.shape[-3:]])
    return h3 * float(np.sum(u * w))


def const_velocity(shape, vc):
    return np.ones((3,) + tuple(shape)) * np.asarray(vc, dtype=float)[:, None, None, None]


# ------------------------------------------------------------------- state
def test_integer_shift_velocity_transports_exactly(orc):
    shape = (16, 12, 10)
    nt = 4
    m = np.array([1, -2, 3])
    h = np.array([TWO_PI / s for s in shape])
    v = const_velocity(shape, m * h * nt)
    rho0 = np.random.default_rng(31).standard_normal(shape)
    P = orc.params(shape, nt, 1e-2)
    rho1 = orc.transport_forward(P, v, rho0)
    expect = np.roll(rho0, shift=tuple(nt * m), axis=(0, 1, 2))
    assert np.abs(rho1 - expect).max() <= 1e-13


def _smooth(x1, x2, x3):
    return np.sin(x1 + 0.2) * np.cos(2 * x2) + 0.5 * np.cos(x3 - x1) + 0.3 * np.sin(x2 + x3)


def test_constant_velocity_converges_fourth_order(orc):
    """rho(x, 1) = rho_T(x - v) for constant v; the only error is the
    interpolation error, which falls like h^4."""
    vc = np.array([0.37, -0.61, 0.23])
    errs = []
    for n in (16, 32, 64):
        shape = (n, n, n)
        x = synth.grid(shape)
        P = orc.params(shape, 4, 1e-2)
        rho1 = orc.transport_forward(P, const_velocity(shape, vc), _smooth(*x))
        errs.append(np.abs(rho1 - _smooth(x[0] - vc[0], x[1] - vc[1], x[2] - vc[2])).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    # D = -dt v / h changes its fractional part with n, so the error constant
    # moves a little between levels; the asymptotic order is 4
    assert min(orders) >= 3.5, (errs, orders)


def test_shear_flow_has_no_time_error(orc):
    """v = (g(x2, x3), 0, 0) gives rho(x, 1) = rho_T(x1 - g, x2, x3); the RK2
    characteristics are exact so refinement in h alone shows 4th order."""
    errs = []
    for n in (16, 32, 64):
        shape = (n, n, n)
        x = synth.grid(shape)
        g = 0.7 * np.sin(x[1]) * np.cos(x[2]) + 0.1
        v = np.stack([g, 0 * g, 0 * g])
        P = orc.params(shape, 3, 1e-2)
        rho1 = orc.transport_forward(P, v, _smooth(*x))
        errs.append(np.abs(rho1 - _smooth(x[0] - g, x[1], x[2])).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 3.7, (errs, orders)


@pytest.mark.slow
def test_smooth_case_second_order_in_time(orc):
    """The smooth divergence-free velocity: error against a fine-step solution
    on the same grid falls like dt^2 (observed order >= 1.8)."""
    shape = (64, 64, 64)
    case = synth.smooth_case(shape)
    ref = orc.transport_forward(orc.params(shape, 64, 1e-2), case["v_true"], case["rhoT"])
    errs = []
    for nt in (2, 4, 8):
        r = orc.transport_forward(orc.params(shape, nt, 1e-2), case["v_true"], case["rhoT"])
        errs.append(np.abs(r - ref).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.8, (errs, orders)


# ----------------------------------------------------------------- adjoint
@pytest.mark.parametrize("iso", [False, True])
def test_adjoint_transport_identity_converges(orc, iso):
    """<S rho0, lam1> = <rho0, S* lam1> holds for the continuous operators;
    the discrete defect (optimise-then-discretise), relative to
    |rho0| |lam1|, shrinks under joint refinement of h and dt: at second
    order in the divergence-free case; in the compressible case the signed
    defect changes sign beyond 64^3, so there it must fall monotonically to
    64^3 and end below 1e-5."""
    defects = []
    for n, nt in ((16, 4), (32, 8), (64, 16)):
        shape = (n, n, n)
        x = synth.grid(shape)
        v = synth.smooth_velocity_divfree(shape) if iso else 0.5 * synth.smooth_velocity_paper(shape)
        rho0 = _smooth(*x)
        lam1 = np.cos(x[0] - 2 * x[2]) + np.sin(x[1]) + _smooth(*x)
        P = orc.params(shape, nt, 1e-2, isochoric=iso)
        rho1 = orc.transport_forward(P, v, rho0)
        lam0 = orc.transport_adjoint(P, v, lam1)
        a, b = inner(rho1, lam1), inner(rho0, lam0)
        defects.append(abs(a - b) / np.sqrt(inner(rho0, rho0) * inner(lam1, lam1)))
    orders = [np.log2(defects[i] / defects[i + 1]) for i in range(2)]
    if iso:
        assert min(orders) >= 1.8, (defects, orders)
    else:
        assert defects[2] < defects[1] < defects[0] and defects[2] < 1e-5, defects


def test_adjoint_conserves_mass_in_the_limit(orc):
    """The adjoint equation is a continuity equation: its integral is
    constant in time; the discrete drift shrinks under refinement."""
    drift = []
    for n, nt in ((16, 4), (32, 8), (64, 16)):
        shape = (n, n, n)
        x = synth.grid(shape)
        v = 0.5 * synth.smooth_velocity_paper(shape)
        lam1 = 1.0 + 0.5 * np.cos(x[0]) * np.sin(x[1] + x[2])
        lam0 = orc.transport_adjoint(orc.params(shape, nt, 1e-2), v, lam1)
        drift.append(abs(lam0.sum() - lam1.sum()) / abs(lam1.sum()))
    assert drift[2] < drift[1] < drift[0], drift


def test_isochoric_adjoint_is_pure_interpolation(orc):
    shape = (16, 16, 16)
    v = synth.smooth_velocity_divfree(shape)
    lam1 = np.random.default_rng(32).standard_normal(shape)
    P = orc.params(shape, 4, 1e-2, isochoric=True)
    lam0 = orc.transport_adjoint(P, v, lam1)
    Da = orc.backtrace(v, 4, -1.0)
    r = lam1
    for _ in range(4):
        r = orc.interp(r, Da)
    assert np.abs(lam0 - r).max() == 0.0


# ------------------------------------------------------- closed forms at v = 0
def _grad_rhoT(shape):
    x = synth.grid(shape)
    return np.stack([np.sin(2 * x[j]) / 3.0 for j in range(3)])


def test_gradient_at_zero_velocity(orc):
    """At v = 0 every transport is the identity, lam = rho_R - rho_T for all t
    and the trapezoid weights sum to one, so g(0) = (rho_R - rho_T) grad rho_T
    (P = I), with grad rho_T known in closed form."""
    shape = (16, 20, 12)
    rhoT = synth.smooth_template(shape)
    rhoR = synth.smooth_random_field(shape, 33, kmax=4)
    P = orc.params(shape, 4, 1e-2)
    g, J, mis = orc.gradient(P, rhoT, rhoR, np.zeros((3,) + shape))
    expect = (rhoR - rhoT)[None] * _grad_rhoT(shape)
    assert np.abs(g - expect).max() <= 1e-13 * np.abs(expect).max()
    assert abs(J - 0.5 * inner(rhoT - rhoR, rhoT - rhoR)) <= 1e-13 * J
    assert abs(mis - 1.0) <= 1e-14


def test_gradient_at_zero_velocity_isochoric(orc):
    shape = (16, 16, 16)
    rhoT = synth.smooth_template(shape)
    rhoR = synth.smooth_random_field(shape, 34, kmax=4)
    P = orc.params(shape, 2, 1e-2, isochoric=True)
    g, _, _ = orc.gradient(P, rhoT, rhoR, np.zeros((3,) + shape))
    expect = orc.leray((rhoR - rhoT)[None] * _grad_rhoT(shape))
    assert np.abs(g - expect).max() <= 1e-13 * np.abs(expect).max()


def test_hessian_at_zero_velocity(orc):
    """At v = 0: rho~(1) = -vt.grad rho_T, lam~ = vt.grad rho_T for all t and
    H vt = beta lap^2 vt + (vt.grad rho_T) grad rho_T; vt is a single mode so
    lap^2 vt = |a|^4 vt."""
    shape = (16, 16, 20)
    x = synth.grid(shape)
    a = np.array([1, -2, 1])
    mode = np.sin(a[0] * x[0] + a[1] * x[1] + a[2] * x[2] + 0.4)
    vt = np.stack([mode, -0.5 * mode, 2.0 * mode])
    beta = 3e-3
    P = orc.params(shape, 4, beta)
    rhoT = synth.smooth_template(shape)
    H = orc.hessian_matvec(P, rhoT, np.zeros((3,) + shape), vt)
    gr = _grad_rhoT(shape)
    s = (vt * gr).sum(0)
    expect = beta * float(a @ a) ** 2 * vt + s[None] * gr
    assert np.abs(H - expect).max() <= 1e-12 * np.abs(expect).max()


def test_hessian_symmetric_and_positive_at_zero(orc):
    shape = (12, 12, 12)
    rng = np.random.default_rng(35)
    P = orc.params(shape, 2, 1e-2)
    rhoT = synth.smooth_template(shape)
    u = synth.smooth_random_field(shape, 36, kmax=3, ncomp=3)
    w = synth.smooth_random_field(shape, 37, kmax=3, ncomp=3)
    v0 = np.zeros((3,) + shape)
    Hu = orc.hessian_matvec(P, rhoT, v0, u)
    Hw = orc.hessian_matvec(P, rhoT, v0, w)
    a, b = inner(Hu, w), inner(u, Hw)
    assert abs(a - b) <= 1e-13 * max(abs(a), 1e-300) * 10
    assert inner(Hu, u) > 0


# --------------------------------------------------------------- refinement
@pytest.mark.slow
def test_gradient_matches_finite_differences_under_refinement(orc):
    """Optimise-then-discretise: <g, vt> is not the derivative of the discrete
    objective, but the defect against a central difference vanishes as h and
    dt are refined together, here at observed order about 3 (2.9 and 3.2
    over 16^3/32^3/48^3 with nt = n/4)."""
    defects = []
    for n, nt in JOINT_LEVELS:
        shape = (n, n, n)
        case = synth.smooth_case(shape)
        P = orc.params(shape, nt, 1e-2)
        rhoR = orc.transport_forward(P, case["v_true"], case["rhoT"])
        v = 0.5 * case["v_true"]
        vt = synth.smooth_random_field(shape, 38, kmax=2, ncomp=3)
        g, _, _ = orc.gradient(P, case["rhoT"], rhoR, v)
        eps = 1e-4
        Jp, _ = orc.objective(P, case["rhoT"], rhoR, v + eps * vt)
        Jm, _ = orc.objective(P, case["rhoT"], rhoR, v - eps * vt)
        fd = (Jp - Jm) / (2 * eps)
        defects.append(abs(fd - inner(g, vt)) / abs(fd))
    o = orders(defects, [n for n, _ in JOINT_LEVELS])
    assert min(o) >= 2.5, (defects, o)


@pytest.mark.slow
def test_hessian_symmetry_defect_converges_at_high_order(orc):
    """Optimise-then-discretise: the discrete GN Hessian is symmetric only in
    the limit. Every piece of it (RK2 in time, eq. (7); trapezoid
    quadrature of b~, eq. (5e); tricubic interpolation) is at least second
    order, so the defect |<Hu,w> - <u,Hw>| / |<Hu,w>| must fall at order >= 2
    under joint refinement (observed about 4.6). A first-order mistake in the
    time levels of the incremental source (eq. (5a)) or in the quadrature
    weights leaves an O(dt) asymmetry: order about 1."""
    r = symmetry_orders(orc)
    assert r["positive"]
    assert min(r["order"]) >= 2.0, r


@pytest.mark.slow
def test_gauss_newton_equals_newton_at_the_true_velocity(orc):
    """At the velocity that generated rho_R (same discretisation) the adjoint
    vanishes, so the Gauss-Newton Hessian is the full Hessian (section II-B):
    central differences of the gradient approach H vt under joint refinement
    at second order or better (observed about 2.6); a first-order slip in
    the time levels of the incremental state gives about 1."""
    r = newton_orders(orc)
    assert min(r["order"]) >= 2.0, r


@pytest.mark.slow
def test_full_newton_matvec_is_the_derivative_of_the_gradient(orc):
    """Away from the true velocity (v = v*/2, lam != 0) the full Hessian of
    eqs. (5a)-(5e), with the source div(lam vt) in the incremental adjoint and
    int lam grad rho~ dt in b~, is the derivative of the reduced gradient:
    central differences of g approach it under joint refinement at second
    order or better (observed about 2.9), while the Gauss-Newton matvec,
    which drops both terms, stays about 16% away. Its symmetry defect falls
    too. A dropped or mis-signed lam term leaves an O(1) defect."""
    r = full_newton_orders(orc)
    assert min(r["newton_order"]) >= 2.0, r
    assert r["newton"][-1] <= 0.01 and min(r["gauss_newton"]) >= 0.1, r
    assert r["symmetry"][-1] < r["symmetry"][0] and max(r["symmetry"]) <= 1e-3, r


@pytest.mark.slow
def test_gradient_and_hessian_are_second_order_in_time(orc):
    """The time discretisation of the whole reduced gradient (eqs. (2b), (3),
    (4)) and of the GN matvec (eqs. (5a), (5c), (5e)) at a fixed v != 0:
    RK2 steps (eq. (7)) and trapezoid sums are second order in dt, so g and
    H vt at nt = 4, 8, 16 approach the nt = 128 solution on the same grid at
    observed order about 2 (1.93 / 1.75 for g, 2.00 / 1.84 for H vt at 32^3;
    the second halving is pulled down by interpolation error that
    accumulates over the steps of the nt = 128 solution). Uniform weights
    1/(nt+1) in b, or the source of the incremental state taken at t^n
    instead of t^{n+1} in the corrector, are first-order mistakes (order
    about 1.05)."""
    r = time_orders(orc)
    assert min(r["g_order"]) >= 1.6 and min(r["H_order"]) >= 1.6, r


# ------------------------------------------------------------- deformation
def test_deformation_integer_shift(orc):
    shape = (12, 16, 10)
    nt = 4
    m = np.array([1, 2, -1])
    h = np.array([TWO_PI / s for s in shape])
    v = const_velocity(shape, m * h * nt)
    u, det, dmin, dmax = orc.deformation(orc.params(shape, nt, 1e-2), v)
    for j in range(3):
        assert np.abs(u[j] + nt * m[j] * h[j]).max() <= 1e-13
    assert abs(dmin - 1) <= 1e-13 and abs(dmax - 1) <= 1e-13


def test_divergence_free_velocity_preserves_volume_in_the_limit(orc):
    errs = []
    for n, nt in ((16, 4), (32, 8), (64, 16)):
        shape = (n, n, n)
        v = synth.smooth_velocity_divfree(shape)
        _, det, dmin, dmax = orc.deformation(orc.params(shape, nt, 1e-2), v)
        errs.append(max(abs(dmin - 1), abs(dmax - 1)))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    # dominated by the O(dt^2) time error of the map
    assert min(orders) >= 1.8 and errs[2] < 5e-3, (errs, orders)


def test_compressible_velocity_changes_volume(orc):
    shape = (16, 16, 16)
    v = synth.smooth_velocity_paper(shape)
    _, det, dmin, dmax = orc.deformation(orc.params(shape, 4, 1e-2), v)
    assert dmin < 0.9 and dmax > 1.1 and dmin > 0
