"""Inputs and probes of the full-size parity check on the 256^3 benchmark
phantom (shared by tests/golden/make_golden.py, which stores the oracle's
values, and tests/test_gpu_fullsize.py, which compares the GPU with them).

The oracle's gradient and Hessian matvec at 256^3 with nt = 16 take minutes
on the host, so their results are stored as scalars: J, the mismatch, norms,
and inner products with seeded white-noise probes (an error e of the GPU
result shows in <e, w> with the size of |e| for white w, at every
frequency). The inputs themselves are cheap and rebuilt by each side."""
import numpy as np

import synth

N = 256
NT = 16
BETA = 1e-3
NPROBES = 4


def _r32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def inputs(oracle, n=N):
    """rho_T (phantom smoothed by the oracle's spectral Gaussian), rho_R (its
    state solve under v_true, nt = 16), v = v_true / 2 and a direction vt,
    all rounded to single precision as the GPU sees them."""
    shape = (n, n, n)
    case = synth.phantom_case(shape, 1003)
    rhoT = _r32(oracle.gauss(case["labels"], case["sigma"]))
    rhoR = _r32(oracle.transport_forward(oracle.params(shape, NT, BETA), case["v_true"], rhoT))
    v = _r32(0.5 * case["v_true"])
    vt = _r32(synth.smooth_random_field(shape, 120, kmax=8, ncomp=3))
    return rhoT, rhoR, v, vt


def probe(n, k):
    """The k-th white-noise probe, a [3][n][n][n] float64 array."""
    return synth.random_field((3, n, n, n), 9000 + k)


def inner(u, w):
    h3 = np.prod([2 * np.pi / m for m in u.shape[-3:]])
    return h3 * float(np.dot(u.ravel(), w.ravel()))
