"""Seeded synthetic inputs for the registration workloads.

This module is shared by the oracle-side tests and the GPU side. It holds
only input recipes (closed-form images, seeded blobs and phantoms, seeded
random velocity fields); it applies none of the registration method's own
operators: no transport, no Leray projection, no spectral smoothing. Where a
workload needs those (the reference image is the template transported by a
known velocity; the phantom is Gaussian-smoothed), each side applies its own
implementation to these raw inputs.

Grid: [0, 2*pi)^3 with x_i = 2*pi*i/N, arrays C-order [N1][N2][N3] (x3
fastest), vector fields [3][N1][N2][N3]. Everything is float64; the caller
casts.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def grid(n):
    """The three coordinate arrays x1, x2, x3 of the periodic grid."""
    n = _shape(n)
    axes = [TWO_PI * np.arange(m) / m for m in n]
    return np.meshgrid(*axes, indexing="ij")


def _shape(n):
    return tuple(int(x) for x in (n if np.ndim(n) else (n, n, n)))


# --------------------------------------------------------------- smooth case
def smooth_template(n):
    """rho_T = (sin^2 x1 + sin^2 x2 + sin^2 x3)/3 (the paper's synthetic template)."""
    x1, x2, x3 = grid(n)
    return (np.sin(x1) ** 2 + np.sin(x2) ** 2 + np.sin(x3) ** 2) / 3.0


def smooth_velocity_divfree(n):
    """v* = (sin x3 cos x2 sin x2, sin x1 cos x3 sin x3, sin x2 cos x1 sin x1).

    Component j does not depend on x_j, so div v* = 0 exactly; max |v*_j| = 1/2."""
    x1, x2, x3 = grid(n)
    return np.stack([
        np.sin(x3) * np.cos(x2) * np.sin(x2),
        np.sin(x1) * np.cos(x3) * np.sin(x3),
        np.sin(x2) * np.cos(x1) * np.sin(x1),
    ])


def smooth_velocity_paper(n):
    """The paper's compressible synthetic velocity (cos x1 sin x2, cos x2 sin x1, cos x1 sin x3)."""
    x1, x2, x3 = grid(n)
    return np.stack([np.cos(x1) * np.sin(x2), np.cos(x2) * np.sin(x1), np.cos(x1) * np.sin(x3)])


# ------------------------------------------------------ random Fourier fields
def _modes(kmax):
    """Integer wave vectors with 1 <= |k|_2 <= kmax, in lexicographic order."""
    r = np.arange(-kmax, kmax + 1)
    k1, k2, k3 = np.meshgrid(r, r, r, indexing="ij")
    k = np.stack([k1.ravel(), k2.ravel(), k3.ravel()], axis=1)
    kk = (k ** 2).sum(1)
    return k[(kk >= 1) & (kk <= kmax * kmax)]


def _trig_field(n, k, coef):
    """Re sum_m coef[c, m] exp(i k_m . x) on the grid, per component c."""
    n = _shape(n)
    spec = np.zeros((coef.shape[0],) + n, dtype=np.complex128)
    idx = tuple((k[:, j] % n[j]) for j in range(3))
    for c in range(coef.shape[0]):
        np.add.at(spec[c], idx, coef[c])
    # numpy's inverse transform carries 1/N; undo it so coefficients are amplitudes
    return np.real(np.fft.ifftn(spec, axes=(1, 2, 3))) * float(np.prod(n))


def random_velocity(n, rng, kmax, max_speed, solenoidal):
    """Random smooth velocity with integer wave numbers 1 <= |k| <= kmax.

    Complex Gaussian coefficients N(0,1) + i N(0,1) per component and mode,
    drawn in one block (real parts, then imaginary parts). With
    solenoidal=True the coefficients are those of a vector potential psi and
    the field is v = curl psi (coefficient i k x psi_k), so div v = 0 by
    construction. The field is scaled so that max_x |v(x)|_2 = max_speed."""
    k = _modes(kmax)
    c = rng.standard_normal((3, len(k))) + 1j * rng.standard_normal((3, len(k)))
    if solenoidal:
        kf = k.astype(np.float64).T  # (3, M)
        c = 1j * np.cross(kf, c, axis=0)
    v = _trig_field(n, k, c)
    speed = np.sqrt((v ** 2).sum(0)).max()
    return v * (max_speed / speed)


# ------------------------------------------------------------------- blobs
def blob_template(n, rng, nblobs=20, sigma_range=(0.1, 0.4), amp_range=(0.5, 1.0)):
    """Sum of Gaussian blobs a*exp(-d^2/(2 sigma^2)) with the per-axis
    minimum-image distance d; draws: centres, then widths, then amplitudes."""
    n = _shape(n)
    centres = rng.uniform(0.0, TWO_PI, size=(nblobs, 3))
    sigmas = rng.uniform(sigma_range[0], sigma_range[1], size=nblobs)
    amps = rng.uniform(amp_range[0], amp_range[1], size=nblobs)
    axes = [TWO_PI * np.arange(m) / m for m in n]
    out = np.zeros(n)
    for b in range(nblobs):
        parts = []
        for j in range(3):
            d = axes[j] - centres[b, j]
            d = (d + np.pi) % TWO_PI - np.pi
            parts.append(np.exp(-d * d / (2.0 * sigmas[b] ** 2)))
        out += amps[b] * parts[0][:, None, None] * parts[1][None, :, None] * parts[2][None, None, :]
    return out


# ----------------------------------------------------------------- phantom
def phantom_labels(n, rng):
    """Six nested axis-aligned ellipsoids painted outer to inner on a zero
    background, with six distinct intensities from {0.1, ..., 1.0}. Draws:
    centre jitter, semi-axis scale, per-shell centre jitter, intensities.
    The caller smooths the result (a Gaussian of width 2 voxels in the
    benchmark workload)."""
    n = _shape(n)
    c0 = np.array([np.pi] * 3) + rng.uniform(-0.1, 0.1, size=3)
    A = np.array([2.2, 2.6, 2.0]) * rng.uniform(0.95, 1.05, size=3)
    jitter = rng.uniform(-0.05, 0.05, size=(6, 3))
    levels = np.round(np.arange(1, 11) / 10.0, 1)
    vals = rng.choice(levels, size=6, replace=False)
    x1, x2, x3 = grid(n)
    out = np.zeros(n)
    for l in range(6):
        c = c0 + (jitter[l] if l > 0 else 0.0)
        a = A * (1.0 - 0.14 * l)
        inside = ((x1 - c[0]) / a[0]) ** 2 + ((x2 - c[1]) / a[1]) ** 2 + ((x3 - c[2]) / a[2]) ** 2 <= 1.0
        out[inside] = vals[l]
    return out


# --------------------------------------------------------------- workloads
def smooth_case(n):
    """Small smooth case: template and divergence-free velocity (no randomness)."""
    return {"rhoT": smooth_template(n), "v_true": smooth_velocity_divfree(n)}


def blob_case(n, seed=1002):
    """Blob template and a solenoidal velocity with |k| <= 4 and max speed 0.5."""
    rng = np.random.default_rng(seed)
    rhoT = blob_template(n, rng)
    v = random_velocity(n, rng, kmax=4, max_speed=0.5, solenoidal=True)
    return {"rhoT": rhoT, "v_true": v}


def blob_case_device(n, seed, device="cuda"):
    """blob_case generated on the host (numpy) and copied to `device` as
    float64 torch tensors (rhoT [n1, n2, n3], v_true [3, n1, n2, n3]); the
    training and test sets of the learned warm start take their pairs from
    here. torch only holds the memory."""
    import torch

    case = blob_case(n, seed)
    return (torch.from_numpy(case["rhoT"]).to(device), torch.from_numpy(case["v_true"]).to(device))


def phantom_case(n, seed=1003):
    """Unsmoothed ellipsoid phantom and a compressible velocity with |k| <= 8
    and max speed 8 cells (8 h radians)."""
    rng = np.random.default_rng(seed)
    labels = phantom_labels(n, rng)
    nn = _shape(n)
    v = random_velocity(n, rng, kmax=8, max_speed=8.0 * TWO_PI / max(nn), solenoidal=False)
    return {"labels": labels, "v_true": v, "sigma": 2.0 * TWO_PI / max(nn)}


def random_field(shape, seed, kind="normal"):
    """Plain seeded random array (for operator tests that need no structure)."""
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal(shape)
    return rng.uniform(-1.0, 1.0, size=shape)


def smooth_random_field(n, seed, kmax=6, ncomp=1, amplitude=1.0):
    """A seeded random trigonometric polynomial with |k| <= kmax (plus a mean)."""
    rng = np.random.default_rng(seed)
    k = _modes(kmax)
    c = (rng.standard_normal((ncomp, len(k))) + 1j * rng.standard_normal((ncomp, len(k)))) / np.sqrt(len(k))
    f = _trig_field(n, k, c) + rng.standard_normal((ncomp, 1, 1, 1))
    f *= amplitude
    return f[0] if ncomp == 1 else f


def displacement(n, seed, max_cells=2.5, kmax=3):
    """A smooth random displacement field in cell units (3, N1, N2, N3),
    scaled so that max |D_j| = max_cells, used to test interpolation away
    from any velocity."""
    D = smooth_random_field(n, seed, kmax=kmax, ncomp=3)
    D -= D.mean(axis=(1, 2, 3), keepdims=True)
    return D * (max_cells / np.abs(D).max())
