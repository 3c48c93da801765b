"""MI355X (gfx950) frequency-domain 3D Helmholtz solves and the adjoint-state
misfit gradient of Da Silva & Herrmann, arXiv:1703.09268.

The compute path lives in ``libhelm.so`` (hand-written HIP kernels behind the
C ABI of ``include/helm.h``); this package only marshals torch tensors into
those entry points.  Importing it does not load the library; the first call
does, and raises if the library has not been built.
"""
from .api import (Grid, SolverOpts, SolveInfo, HelmError, fwi_invert, helm_apply, helm_apply_noalloc, helm_solve,
                  helm_solve_batched, misfit_gradient, misfit_gradient_25d, pde_derivative, version,
                  workspace_bytes, wri_misfit_gradient)
from .autograd import HelmholtzMisfit, helmholtz_misfit

__all__ = ["Grid", "SolverOpts", "SolveInfo", "HelmError", "helm_apply", "helm_apply_noalloc", "helm_solve",
           "helm_solve_batched",
           "misfit_gradient", "pde_derivative", "fwi_invert", "wri_misfit_gradient", "misfit_gradient_25d", "version", "workspace_bytes", "HelmholtzMisfit",
           "helmholtz_misfit"]
