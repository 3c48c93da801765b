"""Oracle: sources, receivers, least-squares misfit and its adjoint-state
gradient in complex128 / float64 (TEST INFRASTRUCTURE; never imported by the
GPU library).

Definitions (paper: Preamble, reduced objective eq. mainprob; Table
derivstuff rows u, V and grad f; Appendix A, eqs. dH and dHadj):

* point source on a grid node (the on-node case of windowed-sinc injection,
  where the interpolation weights reduce to a Kronecker delta):
  ``q_s = S_s e_{p_s} / h^3``;
* receiver sampling ``(P_r u)_r = u_{p_r}``, receivers fixed across sources;
* residual ``r_s = P_r u_s - d_s``, misfit ``f = 1/2 sum_s ||r_s||^2``;
* adjoint field ``v_s = -H^{-H} P_r^T r_s`` (Table derivstuff, row V);
* gradient ``g = sum_s Re(T_s^* v_s) = sum_s Re(omega^2 conj(u_s) * (A^H v_s))``
  (eq. dHadj with T = omega^2 A diag(u)), the derivative of f with respect to
  real m under the real inner product.

``exact_central_difference`` evaluates (f(m + eps e_k) - f(m - eps e_k))/(2
eps) exactly (no cancellation) through the Sherman-Morrison formula for the
rank-one change of H, and ``taylor_remainders`` computes the remainders of the
paper's Taylor test (Validation section).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import operators as ops


def point_source(g: ops.Grid, pos, amp=1.0 + 0.0j) -> np.ndarray:
    q = np.zeros(g.n, dtype=np.complex128)
    q[tuple(int(v) for v in pos)] = amp / g.h ** 3
    return q


def sample(u: np.ndarray, rec: np.ndarray) -> np.ndarray:
    rec = np.asarray(rec)
    return u[rec[:, 0], rec[:, 1], rec[:, 2]]


def sample_adjoint(n, rec: np.ndarray, r: np.ndarray) -> np.ndarray:
    """P_r^T r: scatter-add receiver values onto their nodes."""
    y = np.zeros(n, dtype=np.complex128)
    rec = np.asarray(rec)
    np.add.at(y, (rec[:, 0], rec[:, 1], rec[:, 2]), r)
    return y


def misfit(us, d, rec):
    """f = 1/2 sum_s ||P_r u_s - d_s||^2 and the residuals r_s."""
    rs = [sample(u, rec) - d[s] for s, u in enumerate(us)]
    f = 0.5 * sum(float(np.vdot(r, r).real) for r in rs)
    return f, rs


def mass_apply(x, stencil="7pt", w27=None):
    """A x: identity for the 7-point operator, the 27-point mass
    distribution (real symmetric) for the compact stencil."""
    if stencil == "7pt":
        return x
    return ops.stencil27(x, ops.mass27_weights(w27))


def gradient(g: ops.Grid, us, vs, stencil="7pt", w27=None) -> np.ndarray:
    """sum_s Re(omega^2 conj(u_s) * A^H v_s)."""
    out = np.zeros(g.n, dtype=np.float64)
    for u, v in zip(us, vs):
        out += np.real((g.omega ** 2) * np.conj(u) * mass_apply(v, stencil, w27))
    return out


class LUSolver:
    """Exact discrete solves by sparse LU of the assembled operator."""

    def __init__(self, g, m, stencil="7pt", w27=None):
        self.g = g
        H = ops.assemble(g, m, stencil, w27).tocsc()
        self.lu = spla.splu(H)

    def __call__(self, q, adjoint=False):
        b = np.asarray(q, np.complex128).ravel()
        x = self.lu.solve(b, trans="H" if adjoint else "N")
        return x.reshape(self.g.n)


def misfit_gradient(g: ops.Grid, m, src, rec, d, amp=None, stencil="7pt",
                    w27=None, solve=None):
    """f, g and the forward/adjoint fields for all sources of one frequency.

    ``solve(q, adjoint)`` returns H^{-1} q or H^{-H} q (default: sparse LU).
    """
    solve = solve or LUSolver(g, m, stencil, w27)
    src = np.asarray(src)
    amp = np.ones(len(src), np.complex128) if amp is None else amp
    us = [solve(point_source(g, p, amp[s]), False) for s, p in enumerate(src)]
    f, rs = misfit(us, d, rec)
    vs = [solve(-sample_adjoint(g.n, rec, r), True) for r in rs]
    return f, gradient(g, us, vs, stencil, w27), us, vs


def misfit_gradient_pairs(g: ops.Grid, m, omegas, src, rec, d, amp=None,
                          mask=None, renormalise=False, stencil="7pt",
                          w27=None):
    """f and g summed over (frequency, source) pairs.

    The reduced objective sums the least-squares misfit over every source and
    frequency (Preamble, eq. mainprob: the double sum over i and j); a subset
    of the pairs may be selected (the source/frequency mask of the Software
    Design section), and the stochastic formulation averages over the
    selected pairs, 1/|I| sum_{i in I} f_i (Stochastic FWI section):
    ``renormalise`` divides f and g by the number of selected pairs.

    omegas  angular frequencies, length nfreq (g.omega is not used)
    d       observed data [nfreq][nsrc][nrec]
    amp     source amplitudes [nfreq][nsrc] (default 1)
    mask    bool [nfreq][nsrc] of the selected pairs (default: all)
    Returns (f, g, us, vs) with us/vs dicts keyed by (frequency, source).
    """
    from dataclasses import replace
    src = np.asarray(src)
    nf, ns = len(omegas), len(src)
    amp = np.ones((nf, ns), np.complex128) if amp is None else np.asarray(amp).reshape(nf, ns)
    mask = np.ones((nf, ns), bool) if mask is None else np.asarray(mask, bool).reshape(nf, ns)
    d = np.asarray(d).reshape(nf, ns, -1)
    f_tot = 0.0
    g_tot = np.zeros(g.n, dtype=np.float64)
    us, vs = {}, {}
    for fi, om in enumerate(omegas):
        sel = np.nonzero(mask[fi])[0]
        if len(sel) == 0:
            continue
        gf = replace(g, omega=float(om))
        f, grad, uu, vv = misfit_gradient(gf, m, src[sel], rec, d[fi, sel],
                                          amp=amp[fi, sel], stencil=stencil,
                                          w27=w27)
        f_tot += f
        g_tot += grad
        for k, s in enumerate(sel):
            us[(fi, int(s))] = uu[k]
            vs[(fi, int(s))] = vv[k]
    npair = int(mask.sum())
    if renormalise and npair > 0:
        f_tot /= npair
        g_tot /= npair
    return f_tot, g_tot, us, vs


def exact_central_difference(g: ops.Grid, m, k, eps, us, rs, rec, solve,
                             stencil="7pt", w27=None):
    """(f(m + eps e_k) - f(m - eps e_k)) / (2 eps) without cancellation.

    H(m +- eps e_k) = H +- omega^2 eps a e_k^T with a = A e_k (rank one), so
    u_s^+- = u_s - c_s^+- G with G = H^{-1} a and
    c_s^+- = +-omega^2 eps u_s[k] / (1 +- omega^2 eps G[k]);
    r_s^+- = r_s - c_s^+- p with p = P_r G, and
    f^+ - f^- = sum_s Re((conj(c^-) - conj(c^+)) <p, r_s>)
                + 1/2 (|c^+|^2 - |c^-|^2) ||p||^2.
    """
    k = tuple(int(v) for v in k)
    e = np.zeros(g.n, dtype=np.complex128)
    e[k] = 1.0
    a = mass_apply(e, stencil, w27)
    G = solve(a, False)
    p = sample(G, rec)
    w2e = (g.omega ** 2) * eps
    pp = float(np.vdot(p, p).real)
    diff = 0.0
    for u, r in zip(us, rs):
        cp = w2e * u[k] / (1.0 + w2e * G[k])
        cm = -w2e * u[k] / (1.0 - w2e * G[k])
        pr = np.vdot(p, r)
        diff += float(np.real((np.conj(cm) - np.conj(cp)) * pr)
                      + 0.5 * (abs(cp) ** 2 - abs(cm) ** 2) * pp)
    return diff / (2.0 * eps)


def objective(g, m, src, rec, d, amp=None, stencil="7pt", w27=None):
    """f(m) alone by exact solves (for the Taylor test)."""
    solve = LUSolver(g, m, stencil, w27)
    src = np.asarray(src)
    amp = np.ones(len(src), np.complex128) if amp is None else amp
    us = [solve(point_source(g, p, amp[s]), False) for s, p in enumerate(src)]
    return misfit(us, d, rec)[0]


def taylor_remainders(g, m, dm, src, rec, d, hs, stencil="7pt", w27=None):
    """Zeroth- and first-order Taylor remainders of f along dm:
    |f(m + h dm) - f(m)| and |f(m + h dm) - f(m) - h <grad f, dm>|."""
    f0, grad, _, _ = misfit_gradient(g, m, src, rec, d, stencil=stencil,
                                     w27=w27)
    gd = float(np.sum(grad * dm))
    r0, r1 = [], []
    for h in hs:
        fh = objective(g, m + h * dm, src, rec, d, stencil=stencil, w27=w27)
        r0.append(abs(fh - f0))
        r1.append(abs(fh - f0 - h * gd))
    return np.array(r0), np.array(r1)
