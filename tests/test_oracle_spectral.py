"""Pins of the oracle's FFT and spectral operators against brute force,
numpy's FFT (a library special case) and closed forms on trigonometric
fields (section III-B1 of the paper: Fourier spectral discretisation; the
Leray operator of eq. (4); the biharmonic preconditioner of section III-A)."""
import numpy as np
import pytest

import synth

TWO_PI = 2 * np.pi


def brute_dft3(a, sign=-1):
    """The defining triple sum, as one dense matrix (Kronecker product of the
    three 1D DFT matrices) applied to the flattened array."""
    mats = []
    for n in a.shape:
        j = np.arange(n)
        mats.append(np.exp(sign * 2j * np.pi * np.outer(j, j) / n))
    F = np.kron(np.kron(mats[0], mats[1]), mats[2])
    return (F @ a.ravel()).reshape(a.shape)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 6, 6), (10, 10, 10), (12, 12, 12), (6, 8, 10), (4, 9, 15)])
def test_fft_matches_brute_force(orc, shape):
    rng = np.random.default_rng(11)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert rel(orc.fft3(a, -1), brute_dft3(a, -1)) <= 1e-13
    # inverse: defining sum with +i and 1/N
    assert rel(orc.fft3(a, +1), brute_dft3(a, +1) / a.size) <= 1e-13


@pytest.mark.parametrize("shape", [(32, 32, 32), (48, 48, 48), (30, 20, 18), (64, 16, 24)])
def test_fft_matches_numpy(orc, shape):
    rng = np.random.default_rng(12)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert rel(orc.fft3(a, -1), np.fft.fftn(a)) <= 1e-13
    assert rel(orc.fft3(a, +1), np.fft.ifftn(a)) <= 1e-13


def test_fft_192_radix3(orc):
    """A 192-line (2^6 * 3) transform, the batched workload's largest odd factor."""
    rng = np.random.default_rng(13)
    a = rng.standard_normal((4, 6, 192)) + 1j * rng.standard_normal((4, 6, 192))
    assert rel(orc.fft3(a), np.fft.fftn(a)) <= 1e-13


def _mode(shape, a, phase):
    x = synth.grid(shape)
    arg = a[0] * x[0] + a[1] * x[1] + a[2] * x[2] + phase
    return np.sin(arg), np.cos(arg)


@pytest.mark.parametrize("a", [(1, 0, 0), (0, 2, -1), (3, -2, 5), (-7, 1, 2)])
def test_derivative_and_biharmonic_of_a_mode(orc, a):
    shape = (16, 20, 24)
    s, c = _mode(shape, a, 0.37)
    g = orc.grad(s)
    for j in range(3):
        assert np.abs(g[j] - a[j] * c).max() <= 1e-13 * max(1, abs(a[j]))
    kk = float(np.dot(a, a))
    # round-off in the sampled mode sits in every wavenumber and the even
    # symbols amplify it by up to max|k|^4 (resp. max|k|^2)
    kmax2 = sum((m // 2) ** 2 for m in shape)
    assert np.abs(orc.biharm(s, 1.0) - kk ** 2 * s).max() <= 1e-13 * kk ** 2 + 1e-16 * kmax2 ** 2
    assert np.abs(orc.laplace(s) + kk * s).max() <= 1e-13 * kk + 1e-16 * kmax2
    # inverse biharmonic undoes the biharmonic on zero-mean fields
    assert np.abs(orc.inv_biharm(orc.biharm(s, 0.3), 0.3) - s).max() <= 1e-13
    # Gaussian filter scales a mode by exp(-sigma^2 |a|^2 / 2)
    sig = 0.21
    assert np.abs(orc.gauss(s, sig) - np.exp(-0.5 * sig ** 2 * kk) * s).max() <= 1e-13


def test_nyquist_mode_has_zero_derivative(orc):
    """Odd symbols drop the Nyquist wavenumber: d1 cos(N1 x1 / 2) = 0 on the grid."""
    shape = (16, 8, 8)
    x = synth.grid(shape)
    u = np.cos(shape[0] / 2 * x[0])
    assert np.abs(orc.deriv(u, 0)).max() <= 1e-13
    # the even biharmonic symbol keeps it: lap^2 u = (N/2)^4 u
    assert rel(orc.biharm(u), (shape[0] / 2) ** 4 * u) <= 1e-13


def _inner(u, w):
    h3 = np.prod([TWO_PI / m for m in u.shape[-3:]])
    return h3 * float(np.sum(u * w))


def test_grad_div_are_negative_adjoints(orc):
    shape = (12, 10, 14)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(shape)
    w = rng.standard_normal((3,) + shape)
    lhs = _inner(orc.grad(u), w)
    rhs = -_inner(u, orc.div(w))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0) * 10


def test_leray_projection_invariants(orc):
    shape = (16, 12, 20)
    rng = np.random.default_rng(4)
    v = rng.standard_normal((3,) + shape)
    pv = orc.leray(v)
    # divergence-free to round-off
    assert np.sqrt(_inner(orc.div(pv), orc.div(pv))) <= 1e-13 * np.sqrt(_inner(v, v)) * 10
    # idempotent and self-adjoint
    assert rel(orc.leray(pv), pv) <= 1e-13
    w = rng.standard_normal((3,) + shape)
    a, b = _inner(orc.leray(v), w), _inner(v, orc.leray(w))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)
    # gradients are annihilated; curls are kept
    phi = synth.smooth_random_field(shape, 5, kmax=5)
    assert np.abs(orc.leray(orc.grad(phi))).max() <= 1e-12
    x = synth.grid(shape)
    psi3 = np.sin(x[0] + 2 * x[1]) * np.cos(x[2])
    curl = np.stack([orc.deriv(psi3, 1), -orc.deriv(psi3, 0), np.zeros(shape)])
    assert rel(orc.leray(curl), curl) <= 1e-13


def test_leray_keeps_mean(orc):
    shape = (8, 8, 8)
    v = np.ones((3,) + shape) * np.array([0.5, -1.0, 2.0])[:, None, None, None]
    assert rel(orc.leray(v), v) <= 1e-14


def test_preconditioner_inverts_regularisation(orc):
    """M (beta lap^2 v) = v - mean(v); the isochoric variant adds the projection."""
    shape = (12, 16, 10)
    rng = np.random.default_rng(6)
    v = rng.standard_normal((3,) + shape)
    beta = 1e-2
    z = orc.precond(orc.biharm(v, beta), beta)
    vm = v - v.mean(axis=(1, 2, 3), keepdims=True)
    # the Nyquist planes are kept by the even symbols
    assert rel(z, vm) <= 1e-12
    zi = orc.precond(orc.biharm(v, beta), beta, isochoric=True)
    assert rel(zi, orc.leray(vm)) <= 1e-12


def test_regulariser_parseval(orc):
    """1/2 beta ||lap v||^2 on a single mode: ||lap sin(a.x)||^2 = |a|^4 (2pi)^3 / 2."""
    shape = (16, 16, 16)
    a = (1, 2, -2)
    s, _ = _mode(shape, a, 0.1)
    v = np.stack([s, 0 * s, 2 * s])
    kk = 9.0
    expect = 0.5 * 0.7 * (1 + 4) * kk ** 2 * (TWO_PI ** 3) / 2
    assert abs(orc.regulariser(v, 0.7) - expect) <= 1e-12 * expect


@pytest.mark.parametrize("src,dst", [((24, 24, 24), (16, 16, 16)), ((16, 16, 16), (32, 24, 20))])
def test_resample_preserves_band_limited_fields(orc, src, dst):
    """A trigonometric polynomial with |k_j| < min(N_j, M_j)/2 is reproduced
    exactly on the other grid."""
    a_list = [(1, 2, 3), (0, -5, 1), (7, 0, -4)]
    phases = [0.1, 0.7, -0.4]

    def field(shape):
        x = synth.grid(shape)
        return sum(np.sin(a[0] * x[0] + a[1] * x[1] + a[2] * x[2] + p) for a, p in zip(a_list, phases))

    out = orc.resample(field(src), dst)
    assert np.abs(out - field(dst)).max() <= 1e-12


def test_zero_padding_and_crop(orc):
    """Zero padding (section III-B1) puts the image at the centre offset
    (n - m) // 2 with zeros around it; cropping the same block returns it."""
    img = np.arange(3 * 5 * 4, dtype=np.float64).reshape(3, 5, 4) + 1.0
    out = orc.pad(img, (8, 10, 9))
    assert out.shape == (8, 10, 9)
    assert np.array_equal(out[2:5, 2:7, 2:6], img)
    assert out.sum() == img.sum() and np.count_nonzero(out) == img.size
    assert np.array_equal(orc.crop(out, img.shape), img)
