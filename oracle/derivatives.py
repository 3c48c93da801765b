"""Oracle: linearised modelling (Jacobian), its adjoint, and the Gauss-Newton
and full Hessian-vector products of the least-squares misfit, in
complex128 / float64 (TEST INFRASTRUCTURE; never imported by the GPU library).

Definitions (paper: Table derivstuff, Table derivcosts, the Listing of
PDEfunc cases JACOB_FORW / JACOB_ADJ / HESS_GN / HESS, Appendix A eqs. dU2,
dH, dHadj and DTadj).  For one (frequency, source) pair with field
u = H(m)^{-1} q, H = L + omega^2 A diag(m), real model perturbation dm:

* ``T dm = DH(m)[dm] u = omega^2 A (u * dm)``                  (eq. dH)
* ``T^* z = omega^2 conj(u) * (A^H z)``                         (eq. dHadj)
* field perturbation ``du = -H^{-1} T dm``                       (eq. dU2)
* Jacobian ``J dm = P_r du``                       (Table derivstuff, row J)
* its adjoint, for data y: ``J^* y = Re(T^* v)``, ``v = -H^{-H} P_r^T y``
  (Appendix A, the inner-product derivation; the real part because m is
  real and the data-space inner product is Re(y^H x))
* Gauss-Newton product ``H_GN dm = J^* J dm = Re(T^* w)``,
  ``w = -H^{-H} P_r^T P_r du``   (Table derivstuff, row H_GN: 3 PDE solves)
* full Hessian product of f = 1/2 ||P_r u - d||^2, with the adjoint field
  ``v = -H^{-H} P_r^T r``, r = P_r u - d:
  ``grad^2 f dm = Re(DT^*[dm, du] v) + Re(T^* dv)``, where
  ``DT^*[dm, du] v = omega^2 conj(du) * (A^H v)``               (eq. DTadj)
  and ``dv = H^{-H} (-DH(m)[dm]^H v - P_r^T P_r du)``,
  ``DH(m)[dm]^H v = omega^2 dm * (A^H v)``          (4 PDE solves per pair).

Readings of the paper used here (it is not consistent with itself):
* The Appendix writes dv with ``+ DH(m)[dm]^H v``; differentiating
  ``H^H v = -P_r^T r`` gives ``DH^H v + H^H dv = -P_r^T P_r du``, i.e. a minus
  sign, which is also the sign of Table derivstuff (row DV) and of the HESS
  case of the PDEfunc listing.  The minus sign is used.
* Table derivstuff and the listing write the first term of dv as
  ``DH(m)[dm] V`` (= omega^2 A (dm * v)), the Appendix as ``DH(m)[dm]^H v``
  (= omega^2 dm * (A v)).  They agree for the 7-point operator (A = I); for
  the 27-point operator the derivative of ``H^H v`` needs the latter, which
  is used.
* The HESS_GN case of the listing ends with ``T(U)*dU``; Table derivstuff
  (``T^* H^{-H} P^T P H^{-1} T dm``) and J^* J need the adjoint T^*, which
  is used.

Sums over (frequency, source) pairs follow ``fwi.misfit_gradient_pairs``:
``mask`` selects pairs, ``renormalise`` divides the model-space outputs (J^*,
H_GN, the full Hessian) by the number of selected pairs (the averaged
objective).  ``J dm`` is per pair and is not scaled.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from . import fwi
from . import operators as ops


def born_source(g: ops.Grid, u, dm, stencil="7pt", w27=None):
    """T dm = omega^2 A (u * dm) (eq. dH)."""
    return (g.omega ** 2) * fwi.mass_apply(u * dm, stencil, w27)


def t_adjoint(g: ops.Grid, u, z, stencil="7pt", w27=None):
    """T^* z = omega^2 conj(u) * (A^H z) (eq. dHadj); A is real symmetric."""
    return (g.omega ** 2) * np.conj(u) * fwi.mass_apply(z, stencil, w27)


def _fields(g, m, src, amp, stencil, w27, solve):
    solve = solve or fwi.LUSolver(g, m, stencil, w27)
    src = np.asarray(src)
    amp = np.ones(len(src), np.complex128) if amp is None else np.asarray(amp)
    us = [solve(fwi.point_source(g, p, amp[s]), False) for s, p in enumerate(src)]
    return solve, us


def field_perturbations(g, us, dm, solve, stencil="7pt", w27=None):
    """du_s = -H^{-1} T_s dm for every source (eq. dU2)."""
    return [solve(-born_source(g, u, dm, stencil, w27), False) for u in us]


def jacobian_forward(g: ops.Grid, m, src, rec, dm, amp=None, stencil="7pt",
                     w27=None, solve=None):
    """J dm for every source of one frequency: [nsrc][nrec] complex."""
    solve, us = _fields(g, m, src, amp, stencil, w27, solve)
    dus = field_perturbations(g, us, dm, solve, stencil, w27)
    return np.stack([fwi.sample(du, rec) for du in dus])


def jacobian_adjoint(g: ops.Grid, m, src, rec, y, amp=None, stencil="7pt",
                     w27=None, solve=None):
    """J^* y = sum_s Re(T_s^* v_s), v_s = -H^{-H} P_r^T y_s; y [nsrc][nrec]."""
    solve, us = _fields(g, m, src, amp, stencil, w27, solve)
    out = np.zeros(g.n, dtype=np.float64)
    for s, u in enumerate(us):
        v = solve(-fwi.sample_adjoint(g.n, rec, y[s]), True)
        out += np.real(t_adjoint(g, u, v, stencil, w27))
    return out


def hessian_gn(g: ops.Grid, m, src, rec, dm, amp=None, stencil="7pt",
               w27=None, solve=None):
    """H_GN dm = sum_s Re(T_s^* w_s), w_s = -H^{-H} P_r^T P_r du_s."""
    solve, us = _fields(g, m, src, amp, stencil, w27, solve)
    dus = field_perturbations(g, us, dm, solve, stencil, w27)
    out = np.zeros(g.n, dtype=np.float64)
    for u, du in zip(us, dus):
        w = solve(-fwi.sample_adjoint(g.n, rec, fwi.sample(du, rec)), True)
        out += np.real(t_adjoint(g, u, w, stencil, w27))
    return out


def hessian_full(g: ops.Grid, m, src, rec, d, dm, amp=None, stencil="7pt",
                 w27=None, solve=None):
    """Full Hessian of f = 1/2 sum_s ||P_r u_s - d_s||^2 applied to dm."""
    solve, us = _fields(g, m, src, amp, stencil, w27, solve)
    dus = field_perturbations(g, us, dm, solve, stencil, w27)
    w2 = g.omega ** 2
    out = np.zeros(g.n, dtype=np.float64)
    for s, (u, du) in enumerate(zip(us, dus)):
        r = fwi.sample(u, rec) - d[s]
        v = solve(-fwi.sample_adjoint(g.n, rec, r), True)
        Av = fwi.mass_apply(v, stencil, w27)
        dv = solve(-w2 * dm * Av - fwi.sample_adjoint(g.n, rec, fwi.sample(du, rec)), True)
        out += np.real(w2 * np.conj(du) * Av) + np.real(t_adjoint(g, u, dv, stencil, w27))
    return out


def _pairs(omegas, src, amp, mask):
    src = np.asarray(src)
    nf, ns = len(omegas), len(src)
    amp = np.ones((nf, ns), np.complex128) if amp is None else np.asarray(amp).reshape(nf, ns)
    mask = np.ones((nf, ns), bool) if mask is None else np.asarray(mask, bool).reshape(nf, ns)
    return src, nf, ns, amp, mask


def jacobian_forward_pairs(g, m, omegas, src, rec, dm, amp=None, mask=None,
                           stencil="7pt", w27=None):
    """J dm over (frequency, source) pairs: [nfreq][nsrc][nrec]; rows of
    unselected pairs are zero."""
    src, nf, ns, amp, mask = _pairs(omegas, src, amp, mask)
    out = np.zeros((nf, ns, len(rec)), np.complex128)
    for fi, om in enumerate(omegas):
        sel = np.nonzero(mask[fi])[0]
        if len(sel):
            out[fi, sel] = jacobian_forward(replace(g, omega=float(om)), m, src[sel], rec, dm,
                                            amp[fi, sel], stencil, w27)
    return out


def _model_space_pairs(fn, g, m, omegas, src, amp, mask, renormalise, per_freq):
    src, nf, ns, amp, mask = _pairs(omegas, src, amp, mask)
    out = np.zeros(g.n, dtype=np.float64)
    for fi, om in enumerate(omegas):
        sel = np.nonzero(mask[fi])[0]
        if len(sel):
            out += fn(replace(g, omega=float(om)), src[sel], amp[fi, sel], per_freq(fi, sel))
    npair = int(mask.sum())
    if renormalise and npair > 0:
        out /= npair
    return out


def jacobian_adjoint_pairs(g, m, omegas, src, rec, y, amp=None, mask=None,
                           renormalise=False, stencil="7pt", w27=None):
    """J^* y summed over the selected pairs; y [nfreq][nsrc][nrec]."""
    y = np.asarray(y).reshape(len(omegas), len(src), -1)
    return _model_space_pairs(
        lambda gf, s, a, yy: jacobian_adjoint(gf, m, s, rec, yy, a, stencil, w27),
        g, m, omegas, src, amp, mask, renormalise, lambda fi, sel: y[fi, sel])


def hessian_gn_pairs(g, m, omegas, src, rec, dm, amp=None, mask=None,
                     renormalise=False, stencil="7pt", w27=None):
    return _model_space_pairs(
        lambda gf, s, a, _: hessian_gn(gf, m, s, rec, dm, a, stencil, w27),
        g, m, omegas, src, amp, mask, renormalise, lambda fi, sel: None)


def hessian_full_pairs(g, m, omegas, src, rec, d, dm, amp=None, mask=None,
                       renormalise=False, stencil="7pt", w27=None):
    d = np.asarray(d).reshape(len(omegas), len(src), -1)
    return _model_space_pairs(
        lambda gf, s, a, dd: hessian_full(gf, m, s, rec, dd, dm, a, stencil, w27),
        g, m, omegas, src, amp, mask, renormalise, lambda fi, sel: d[fi, sel])


def forward_data(g, m, src, rec, amp=None, stencil="7pt", w27=None):
    """F(m) = P_r u(m) for every source (exact solves): [nsrc][nrec]."""
    _, us = _fields(g, m, src, amp, stencil, w27, None)
    return np.stack([fwi.sample(u, rec) for u in us])
