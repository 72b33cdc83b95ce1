"""MI355X (gfx950) semi-Lagrangian Gauss-Newton-Krylov diffeomorphic
registration: the HIP library behind include/reg.h and its Python binding.

The hot path (interpolation, characteristics, transport solves, spectral
operators, gradient, Gauss-Newton Hessian, preconditioner and the solver) runs
in hand-written HIP kernels in ``libreg.so``; PyTorch supplies device memory
and streams only.
"""
from .reg import (  # noqa: F401
    Context,
    RegError,
    REG_OK,
    REG_EINVAL,
    REG_ELINESEARCH,
    REG_ENONFINITE,
    SPEC_BIHARM,
    SPEC_GAUSS,
    SPEC_INVBIHARM,
    SPEC_LERAY,
    lib,
    reg_default_params,
    reg_params,
    reg_report,
    reg_workspace_size,
)
