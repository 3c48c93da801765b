"""Differentiable least-squares misfit f(m) behind ``torch.autograd.Function``.

Forward: one multi-source (and multi-frequency) forward solve (``misfit_gradient`` with
HELM_MG_FORWARD_ONLY), keeping the fields u_s as their FP64 outer iterates
(HELM_MG_U_FP64), so the receiver residual formed again in backward is as
accurate as the one formed inside a single misfit_gradient call.  Backward: the adjoint solves
and the hand-written gradient kernel (``misfit_gradient`` with
HELM_MG_REUSE_U), g = sum_s Re(omega^2 conj(u_s) * A^H v_s) with
v_s = -H^{-H} P_r^T (P_r u_s - d_s) (paper: Table derivstuff, rows V and
grad f; Appendix A, eq. dHadj).  The map is real m -> real f, so there is no
complex (Wirtinger) convention to choose.
"""
from __future__ import annotations

import numpy as np
import torch

from .api import Grid, SolverOpts, misfit_gradient


class HelmholtzMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m: torch.Tensor, grid: Grid, omega, src, rec, d: torch.Tensor,
                opts: SolverOpts = None, src_amp=None, mask=None, renormalise: bool = False):
        m_c = m.detach().contiguous()
        nfreq = int(np.atleast_1d(np.asarray(omega)).size)
        u_store = torch.empty((nfreq, len(src)) + tuple(int(a) for a in grid.n),
                              dtype=torch.complex128, device=m.device)
        kw = dict(src_amp=src_amp, mask=mask, renormalise=renormalise, opts=opts)
        f, _, infos = misfit_gradient(grid, m_c, omega, src, rec, d, u_store=u_store,
                                      forward_only=True, u_fp64=True, **kw)
        ctx.save_for_backward(m_c)
        ctx.u_store = u_store
        ctx.args = (grid, omega, src, rec, d, kw)
        ctx.forward_infos = infos
        return torch.tensor(f, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        (m_c,) = ctx.saved_tensors
        grid, omega, src, rec, d, kw = ctx.args
        _, g, _ = misfit_gradient(grid, m_c, omega, src, rec, d, u_store=ctx.u_store,
                                  reuse_u=True, u_fp64=True, **kw)
        if not (grad_f.numel() == 1 and float(grad_f) == 1.0):
            g = g * grad_f.to(g.dtype)
        return g, None, None, None, None, None, None, None, None, None


def helmholtz_misfit(m, grid, omega, src, rec, d, opts=None, src_amp=None, mask=None,
                     renormalise=False):
    """f(m) = 1/2 sum over the selected (frequency, source) pairs of
    ||P_r H_f(m)^{-1} q_fs - d_fs||^2 (divided by the number of selected pairs
    with renormalise), differentiable in m.  omega: one angular frequency or
    a sequence; d: [nfreq][nsrc][nrec] complex device tensor."""
    return HelmholtzMisfit.apply(m, grid, omega, src, rec, d, opts, src_amp, mask, renormalise)
