"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

TWO_PI = 2 * np.pi

# Tolerances (relative L2 unless stated), GPU against the FP64 oracle on the
# same (already rounded) inputs. Double-precision kernels differ from the
# oracle only by summation order; single-precision ones by FP32 rounding in
# the kernels' own arithmetic.
TOL = {
    ("interp", 1): 1e-12, ("interp", 0): 1e-6,
    ("backtrace", 1): 1e-12, ("backtrace", 0): 1e-6,
    ("transport", 1): 1e-12, ("transport", 0): 1e-5,
    ("spectral", 1): 1e-12, ("spectral", 0): 1e-6,
    ("scalar", 1): 1e-12, ("scalar", 0): 1e-5,
    ("det", 1): 1e-10, ("det", 0): 1e-4,
}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def to_dev(x, ctx):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=ctx.device, dtype=ctx.dtype).contiguous()


def to_vel(x, ctx):
    """A velocity-space tensor (always float64)."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device=ctx.device).contiguous()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy()


def rounded(x, prec):
    """The inputs both sides see: cast to the GPU precision, then to float64."""
    return np.asarray(x, dtype=np.float64 if prec else np.float32).astype(np.float64)


def say(msg):
    print(msg, flush=True)


def unit_roundoff(prec):
    return 2.0 ** -53 if prec else 2.0 ** -24


def biharm_amp(shape):
    """sqrt(mean_k |k|^8) over the grid's wavenumbers."""
    ks = [np.fft.fftfreq(n, 1.0 / n) for n in shape]
    k2 = ks[0][:, None, None] ** 2 + ks[1][None, :, None] ** 2 + ks[2][None, None, :] ** 2
    return float(np.sqrt(np.mean(k2 ** 4)))


def deriv_bound(shape, prec, fields, out_ref, safety=4.0):
    """Relative-L2 error bound of a first derivative (or a sum of them) in
    floating point: round-off of the line transform (relative size ~u per
    mode, white across the spectrum) is multiplied by k_j, so its norm grows
    to u sqrt(sum_j mean_k k_j^2 |f_j|^2) for fields f_j differentiated along
    axis j (a dict axis -> field), against the result's norm. It reaches
    u n / sqrt(12) per axis of n points, so long lines and smooth inputs need
    more than a fixed bar in single precision."""
    acc = 0.0
    for j, f in fields.items():
        kj = np.fft.fftfreq(shape[j], 1.0 / shape[j])
        acc += float(np.mean(kj ** 2)) * float(np.sum(np.asarray(f, dtype=np.float64) ** 2))
    bound = safety * unit_roundoff(prec) * np.sqrt(acc) / np.linalg.norm(np.ravel(out_ref))
    return max(TOL[("spectral", prec)], bound)


def biharm_bound(shape, prec, scale_v_norm, out_norm, safety=4.0):
    """Relative-L2 error bound of a result that contains scale*lap^2 v.

    Round-off of the forward transform (relative size ~u per mode, white
    across the spectrum) is multiplied by |k|^4 in every mode, so its norm
    grows to u sqrt(mean_k |k|^8) scale |v| against a result of norm out_norm;
    the bound is that ratio times a safety factor."""
    return safety * unit_roundoff(prec) * biharm_amp(shape) * scale_v_norm / out_norm


def biharm_fp32_bound(shape, v, out_ref, safety=4.0):
    """biharm_bound for out_ref = lap^2 v computed in single precision."""
    return biharm_bound(shape, 0, np.linalg.norm(np.ravel(v)), np.linalg.norm(np.ravel(out_ref)), safety)
