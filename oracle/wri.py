"""Oracle: Wavefield Reconstruction Inversion, the paper's penalty method
(TEST INFRASTRUCTURE; never imported by the GPU library).

Paper: Penalty Method subsection (eqs. wri and wrifieldeq) and Appendix B
(derivative expressions for WRI).  For a fixed model m the field u(m)
minimises

    phi(m, u) = 1/2 ||P_r u - d||^2 + lambda^2 / 2 ||H(m) u - q||^2,

i.e. solves the normal equations of the stacked least-squares problem
[P_r; lambda H] u = [d; lambda q],

    (P_r^T P_r + lambda^2 H^H H) u = P_r^T d + lambda^2 H^H q,

the objective is f(m) = phi(m, u(m)), and by variable projection its
gradient is lambda^2 T(m, u)^* (H u - q), with T^* z = omega^2 conj(u) *
(A^H z) (real part, real m) as for the reduced objective.  Summed over the
selected (frequency, source) pairs like the reduced misfit (and divided by
their number with renormalise).  The normal equations are solved here by
sparse LU: the plain definition, no iteration.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fwi
from . import operators as ops


def selection(n, rec) -> sp.csr_matrix:
    """P_r as a sparse (nrec x N) matrix of on-node samples."""
    rec = np.asarray(rec)
    lin = (rec[:, 0] * n[1] + rec[:, 1]) * n[2] + rec[:, 2]
    N = int(np.prod(n))
    return sp.csr_matrix((np.ones(len(rec)), (np.arange(len(rec)), lin)), shape=(len(rec), N))


def wri_fields(g: ops.Grid, m, src, rec, d, lam, amp=None, stencil="7pt", w27=None):
    """u(m) for every source of one frequency (d: [nsrc][nrec])."""
    H = ops.assemble(g, m, stencil, w27).tocsc()
    P = selection(g.n, rec).astype(np.complex128)
    Hh = H.conj().T.tocsc()
    G = (P.T @ P + lam ** 2 * (Hh @ H)).tocsc()
    lu = spla.splu(G)
    amp = np.ones(len(src), np.complex128) if amp is None else amp
    us, qs = [], []
    for s, p in enumerate(np.asarray(src)):
        q = fwi.point_source(g, p, amp[s]).ravel()
        rhs = P.T @ np.asarray(d[s], np.complex128) + lam ** 2 * (Hh @ q)
        us.append(lu.solve(rhs).reshape(g.n))
        qs.append(q.reshape(g.n))
    return us, qs, H, P


def wri_misfit_gradient(g: ops.Grid, m, src, rec, d, lam, amp=None, stencil="7pt", w27=None):
    """f = sum_s phi(m, u_s(m)) and grad f = sum_s lambda^2 Re(omega^2
    conj(u_s) * A^H (H u_s - q_s)) for one frequency; also the fields."""
    us, qs, H, P = wri_fields(g, m, src, rec, d, lam, amp, stencil, w27)
    f = 0.0
    grad = np.zeros(g.n)
    for s, (u, q) in enumerate(zip(us, qs)):
        rd = P @ u.ravel() - np.asarray(d[s])
        e = (H @ u.ravel() - q.ravel()).reshape(g.n)
        f += 0.5 * float(np.vdot(rd, rd).real) + 0.5 * lam ** 2 * float(np.vdot(e, e).real)
        grad += lam ** 2 * np.real(g.omega ** 2 * np.conj(u) * fwi.mass_apply(e, stencil, w27))
    return f, grad, us


def wri_misfit_gradient_pairs(g: ops.Grid, m, omegas, src, rec, d, lam, amp=None, mask=None,
                              renormalise=False, stencil="7pt", w27=None):
    """Sum over the selected (frequency, source) pairs, as fwi.misfit_gradient_pairs."""
    src = np.asarray(src)
    nf, ns = len(omegas), len(src)
    amp = np.ones((nf, ns), np.complex128) if amp is None else np.asarray(amp).reshape(nf, ns)
    mask = np.ones((nf, ns), bool) if mask is None else np.asarray(mask, bool).reshape(nf, ns)
    d = np.asarray(d).reshape(nf, ns, -1)
    f_tot, g_tot, us = 0.0, np.zeros(g.n), {}
    for fi, om in enumerate(omegas):
        sel = np.nonzero(mask[fi])[0]
        if len(sel) == 0:
            continue
        f, grad, uu = wri_misfit_gradient(replace(g, omega=float(om)), m, src[sel], rec, d[fi, sel], lam,
                                          amp[fi, sel], stencil, w27)
        f_tot += f
        g_tot += grad
        for k, s in enumerate(sel):
            us[(fi, int(s))] = uu[k]
    npair = int(mask.sum())
    if renormalise and npair:
        f_tot /= npair
        g_tot /= npair
    return f_tot, g_tot, us
