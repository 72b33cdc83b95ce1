"""Pins of the oracle's periodic tricubic Lagrange interpolation (sections
III-B2 and III-C2 of the paper: the interpolation at semi-Lagrangian points
uses a 4^3 = 64-point stencil) and of the RK2 departure points (eq. (6))."""
import numpy as np
import pytest

import synth

TWO_PI = 2 * np.pi


def lagrange_by_polyfit(vals, t):
    """The cubic through (-1, v0), (0, v1), (1, v2), (2, v3) evaluated at t,
    obtained from numpy's least-squares polynomial fit (exact for 4 points)."""
    c = np.polyfit(np.array([-1.0, 0.0, 1.0, 2.0]), vals, 3)
    return np.polyval(c, t)


def test_interp_matches_separable_library_fit(orc):
    """Tensor-product cubic interpolation done axis by axis with np.polyfit,
    on a tiny ragged grid with displacements that wrap around the boundary."""
    shape = (6, 7, 8)
    rng = np.random.default_rng(21)
    f = rng.standard_normal(shape)
    D = rng.uniform(-3.5, 3.5, size=(3,) + shape)
    out = orc.interp(f, D)
    for p in rng.choice(f.size, size=40, replace=False):
        i = np.unravel_index(p, shape)
        s = [i[j] + D[j][i] for j in range(3)]
        m = [int(np.floor(x)) for x in s]
        t = [x - mm for x, mm in zip(s, m)]
        # along x3, then x2, then x1
        plane = np.empty((4, 4))
        for a in range(4):
            for b in range(4):
                row = [f[(m[0] + a - 1) % shape[0], (m[1] + b - 1) % shape[1], (m[2] + c - 1) % shape[2]]
                       for c in range(4)]
                plane[a, b] = lagrange_by_polyfit(np.array(row), t[2])
        line = np.array([lagrange_by_polyfit(plane[a], t[1]) for a in range(4)])
        expect = lagrange_by_polyfit(line, t[0])
        assert abs(out[i] - expect) <= 1e-12 * max(1.0, abs(expect))


def test_cubic_polynomials_are_reproduced(orc):
    """Any polynomial of degree <= 3 per axis is reproduced where the stencil
    does not wrap."""
    shape = (16, 16, 16)
    idx = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    coef = np.random.default_rng(22).standard_normal((4, 4, 4))

    def poly(z1, z2, z3):
        out = 0.0
        for a in range(4):
            for b in range(4):
                for c in range(4):
                    out = out + coef[a, b, c] * (z1 / 8) ** a * (z2 / 8) ** b * (z3 / 8) ** c
        return out

    f = poly(*idx)
    D = synth.displacement(shape, 23, max_cells=0.99)
    out = orc.interp(f, D)
    inner = (slice(2, 13),) * 3  # i in [2, 12], |D| < 1 keeps m-1..m+2 inside [0, 15]
    exact = poly(idx[0] + D[0], idx[1] + D[1], idx[2] + D[2])
    assert np.abs(out[inner] - exact[inner]).max() <= 1e-12 * np.abs(exact[inner]).max()


def test_integer_displacement_is_an_exact_shift(orc):
    shape = (8, 10, 12)
    f = np.random.default_rng(24).standard_normal(shape)
    m = (2, -3, 5)
    D = np.stack([np.full(shape, float(x)) for x in m])
    out = orc.interp(f, D)
    assert np.array_equal(out, np.roll(f, shift=(-m[0], -m[1], -m[2]), axis=(0, 1, 2)))


def test_constant_field_is_kept(orc):
    shape = (9, 10, 11)
    D = synth.displacement(shape, 25, max_cells=4.0)
    out = orc.interp(np.full(shape, 1.75), D)
    assert np.abs(out - 1.75).max() <= 1e-14


def test_fourth_order_convergence(orc):
    """Error of interpolating a smooth periodic function at a fixed set of
    physical points falls like h^4 (observed order >= 3.8 over 32 -> 64 -> 128)."""
    def f_exact(x1, x2, x3):
        return np.exp(np.sin(x1)) * np.cos(2 * x2 + 0.3) + np.sin(x3 - x1)

    errs = []
    for n in (32, 64, 128):
        shape = (n, n, 4)
        x = synth.grid(shape)
        # physical displacement (radians), the same function of x for every n
        dphys = np.stack([0.3 * np.sin(x[1]), 0.25 * np.cos(x[0]), 0 * x[0]])
        h = np.array([TWO_PI / m for m in shape])[:, None, None, None]
        D = dphys / h
        f = f_exact(*x)
        out = orc.interp(f, D)
        errs.append(np.abs(out - f_exact(x[0] + dphys[0], x[1] + dphys[1], x[2])).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 3.8, (errs, orders)


def test_interp_transpose_identity(orc):
    """<I_D f, g> = <f, I_D^T g> for the scatter-add transpose."""
    shape = (6, 8, 7)
    rng = np.random.default_rng(26)
    f = rng.standard_normal(shape)
    g = rng.standard_normal(shape)
    D = rng.uniform(-2, 2, size=(3,) + shape)
    a = float(np.sum(orc.interp(f, D) * g))
    b = float(np.sum(f * orc.interp_transpose(g, D)))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


# ------------------------------------------------------------------- backtrace
def test_backtrace_constant_velocity(orc):
    """Constant v: both RK2 stages see the same velocity, D = -dt v / h."""
    shape = (8, 12, 10)
    nt = 4
    vc = np.array([0.3, -1.1, 2.0])
    v = np.ones((3,) + shape) * vc[:, None, None, None]
    for sign in (1.0, -1.0):
        D = orc.backtrace(v, nt, sign)
        for j in range(3):
            h = TWO_PI / shape[j]
            assert np.abs(D[j] + sign * vc[j] / nt / h).max() <= 1e-13 * max(1, abs(vc[j]) / nt / h)


def test_backtrace_shear_flow_is_exact(orc):
    """v = (g(x2, x3), 0, 0): the first stage moves only along x1, where v is
    constant, so v(X*) = v(x) exactly and D1 = -dt g / h1."""
    shape = (16, 12, 10)
    x = synth.grid(shape)
    g = 0.8 * np.sin(x[1]) * np.cos(x[2]) + 0.2
    v = np.stack([g, 0 * g, 0 * g])
    D = orc.backtrace(v, 4)
    h1 = TWO_PI / shape[0]
    assert np.abs(D[0] + 0.25 * g / h1).max() <= 1e-13
    assert np.abs(D[1]).max() == 0 and np.abs(D[2]).max() == 0


def test_backtrace_second_order_in_dt(orc):
    """RK2 departure points against the exact characteristic of a smooth
    velocity (integrated with many small RK4 steps): error ~ dt^3 per step."""
    shape = (32, 32, 32)
    v = synth.smooth_velocity_divfree(shape)
    x = np.stack(synth.grid(shape))

    def vel(X):
        x1, x2, x3 = X
        return np.stack([np.sin(x3) * np.cos(x2) * np.sin(x2), np.sin(x1) * np.cos(x3) * np.sin(x3),
                         np.sin(x2) * np.cos(x1) * np.sin(x1)])

    errs = []
    for nt in (2, 4, 8):
        dt = 1.0 / nt
        # exact: integrate dX/ds = -v(X) from X = x for time dt
        X = x.copy()
        m = 64
        hs = dt / m
        for _ in range(m):
            k1 = -vel(X)
            k2 = -vel(X + 0.5 * hs * k1)
            k3 = -vel(X + 0.5 * hs * k2)
            k4 = -vel(X + hs * k3)
            X = X + hs / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        h = TWO_PI / 32
        D = orc.backtrace(v, nt)
        errs.append(np.abs(x + h * D - X).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    # local error of a 2nd-order step is O(dt^3); interpolation error (h^4)
    # is well below it at this resolution
    assert min(orders) >= 2.7, (errs, orders)
