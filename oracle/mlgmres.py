"""Oracle: the ML-GMRES preconditioner and solve in complex128
(TEST INFRASTRUCTURE; never imported by the GPU library).

Follows the paper's multi-level recursive preconditioner section: a standard
multigrid V-cycle (algorithm "Standard multigrid V-cycle") whose smoother is
GMRES with an identity preconditioner, whose coarse problem is the same
Helmholtz problem on the coarser grid solved by FGMRES and preconditioned by
the same V-cycle one level down, with linear interpolation as prolongation
and its adjoint as restriction; three grids (h, 2h, 4h), the coarsest solved
by plain GMRES; the outer solver is FGMRES with 5 inner iterations to a
relative residual of 1e-6.  Memory parameters (k_so, k_si, k_co, k_ci) =
(3, 5, 3, 5): smoother GMRES(3 cycles, 5 steps), coarse (F)GMRES(3, 5).

Readings where the paper is open or garbled:
* coarse grid: n_c = floor(n_f/2) + 1 nodes per axis, coarse node I at fine
  node 2I (fine nodes past the end are zero);
* coarse operator: the same discretisation re-built at spacing 2h, same
  omega, layer profile evaluated at the fine coordinates 2I and 2I +- 1;
  coarse model by injection m_c(I) = m_f(min(2I, n_f - 1));
* restriction R = P^T / 8 (the adjoint of P in the h^3-weighted inner
  product; the unscaled transpose would weight the correction by 8);
* the V-cycle starts from x = 0, the right-hand side restriction the
  algorithm lists (b_c = R b_f) is not used by any later step and is
  skipped, and the interpolated correction is added to the smoothed iterate;
* inner solves run fixed iteration counts with no tolerance test.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import operators as ops
from .krylov import gmres, fgmres


# ----------------------------------------------------------------------------
# transfer operators
# ----------------------------------------------------------------------------

def interp_matrix_1d(nf: int) -> np.ndarray:
    """Dense 1D linear interpolation P (nf x nc), nc = nf//2 + 1:
    even fine node 2I -> coarse I (weight 1); odd fine node 2I+1 -> 1/2 from
    coarse I and 1/2 from coarse I+1."""
    nc = nf // 2 + 1
    P = np.zeros((nf, nc))
    for i in range(nf):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, (i - 1) // 2] = 0.5
            P[i, (i + 1) // 2] = 0.5
    return P


def _apply_axes(x, mats):
    y = x
    for a, M in enumerate(mats):
        y = np.moveaxis(np.tensordot(M, np.moveaxis(y, a, 0), axes=(1, 0)), 0, a)
    return y


def prolong(xc: np.ndarray, nf) -> np.ndarray:
    """P x_c: tensor product of 1D linear interpolation."""
    return _apply_axes(np.asarray(xc), [interp_matrix_1d(n) for n in nf])


def restrict(rf: np.ndarray) -> np.ndarray:
    """R r_f = (1/8) P^T r_f."""
    mats = [interp_matrix_1d(n).T for n in rf.shape]
    return _apply_axes(np.asarray(rf), mats) / 8.0


def inject_model(mf: np.ndarray) -> np.ndarray:
    """Coarse model by injection: m_c(I) = m_f(min(2I, n_f - 1))."""
    sl = []
    for n in mf.shape:
        nc = n // 2 + 1
        sl.append(np.minimum(2 * np.arange(nc), n - 1))
    return mf[np.ix_(*sl)].copy()


# ----------------------------------------------------------------------------
# hierarchy and V-cycle
# ----------------------------------------------------------------------------

@dataclass
class MLOptions:
    ks_o: int = 3   # smoother restart cycles
    ks_i: int = 5   # smoother Krylov dimension
    kc_o: int = 3   # coarse-solve restart cycles
    kc_i: int = 5   # coarse-solve Krylov dimension
    levels: int = 3  # number of grids
    k_outer: int = 5  # outer FGMRES Krylov dimension


class Hierarchy:
    """Grids, models and operators of all levels for one (m, omega)."""

    def __init__(self, g: ops.Grid, m: np.ndarray, opts: MLOptions,
                 stencil="7pt", w27=None, adjoint=False):
        self.opts = opts
        self.adjoint = adjoint
        self.grids = [g]
        self.models = [np.asarray(m, np.float64)]
        for _ in range(opts.levels - 1):
            self.grids.append(ops.coarsen(self.grids[-1]))
            self.models.append(inject_model(self.models[-1]))
        self.stencil = stencil
        self.w27 = w27

    def A(self, lvl):
        g, m = self.grids[lvl], self.models[lvl]
        st, w27, adj = self.stencil, self.w27, self.adjoint

        def op(x):
            return ops.apply(g, m, x, adjoint=adj, stencil=st, w27=w27)
        return op

    def smooth(self, lvl, b, x0):
        o = self.opts
        x, _ = gmres(self.A(lvl), b, x0=x0, k=o.ks_i, cycles=o.ks_o, tol=None)
        return x

    def vcycle(self, lvl, b):
        """One V-cycle for H_lvl x = b starting from x = 0."""
        o = self.opts
        x = self.smooth(lvl, b, None)                     # pre-smooth
        r = b - self.A(lvl)(x)                            # residual
        rc = restrict(r)                                  # restrict
        if lvl + 1 == o.levels - 1:                       # coarsest grid
            xc, _ = gmres(self.A(lvl + 1), rc, k=o.kc_i, cycles=o.kc_o,
                          tol=None)
        else:                                             # recursive coarse
            xc, _ = fgmres(self.A(lvl + 1), rc,
                           M=lambda v: self.vcycle(lvl + 1, v),
                           k=o.kc_i, cycles=o.kc_o, tol=None)
        x = x + prolong(xc, self.grids[lvl].n)            # correct
        return self.smooth(lvl, b, x)                     # post-smooth


def mlgmres_solve(g: ops.Grid, m, q, tol=1e-6, max_cycles=50,
                  opts: MLOptions = None, stencil="7pt", w27=None,
                  adjoint=False, x0=None, history=None):
    """Outer FGMRES(k_outer) on H u = q (or H^H u = q) preconditioned by the
    level-0 V-cycle; restarts until the relative residual <= tol."""
    opts = opts or MLOptions()
    if opts.levels < 2:
        raise ValueError("ML-GMRES needs at least two grids")
    hier = Hierarchy(g, m, opts, stencil, w27, adjoint)
    return fgmres(hier.A(0), q, M=lambda v: hier.vcycle(0, v), x0=x0,
                  k=opts.k_outer, cycles=max_cycles, tol=tol, history=history)


def workspace_vectors(opts: MLOptions) -> float:
    """The paper's peak-memory bound, in vectors of fine size N:
    (2k+6) + max((k_si+5), (2k_ci+6)/8 + max((k_si+5)/8, (2k_ci+6)/64))."""
    k, ksi, kci = opts.k_outer, opts.ks_i, opts.kc_i
    return (2 * k + 6) + max(ksi + 5, (2 * kci + 6) / 8.0
                             + max((ksi + 5) / 8.0, (2 * kci + 6) / 64.0))
