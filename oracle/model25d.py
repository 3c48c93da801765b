"""Oracle: 2.5D modelling, misfit and gradient (TEST INFRASTRUCTURE; never
imported by the GPU library).

Paper: the 2.5D subsection.  For a model invariant along y, a Fourier
transform in y turns the 3D Helmholtz equation into the 2D equations

    H(k_y) u~ = S delta(x - x_s) delta(z - z_s),
    H(k_y) = d_xx + d_zz + omega^2 m(x, z) - k_y^2,      k_y >= 0,

and the 3D field is recovered as

    u(x, y, z) = (1/pi) int_0^K u~_{k_y}(x, z) cos(k_y (y - y_s)) dk_y,

the integral cut at K = min(p k_c, k_nyq), k_c = omega / v_min (the critical
wavenumber), k_nyq = pi / dy, and evaluated by Gauss-Legendre quadrature:
u ~ sum_i w_i u~_{k_i} cos(k_i (y - y_s)) with the 1/pi folded into w_i.
Here dy = h (the grid spacing), p and v_min are inputs (the paper takes
p >= 1, p ~ 1), so the rule does not depend on the model.

Discretisation (as the 3D operator of this repository): the 2D grid is a 3D
grid with one node along its first axis; its (second, third) axes carry the
paper's (x, z); each axis has the layer-stretched 3-point row of the 3D
operator; the point source is amp e_s / h^2 (the 2D discrete delta).
Sources and receivers sit on nodes of the plane, each with its own
coordinate along the invariant axis (y_s, y_r, in metres).

Misfit over the (frequency, source) pairs, with c_{s,i,r} = w_i cos(k_i (y_r
- y_s)):  d_s = sum_i c_{s,i} * P u~_{s,i},  f = 1/2 sum_s ||d_s - d_obs,s||^2,
and its gradient (derivative of each 2D equation in m is omega^2):
    g = sum_{s,i} Re(omega^2 conj(u~_{s,i}) * v_{s,i}),
    v_{s,i} = -H(k_i)^{-H} P^T (c_{s,i} * r_s),     r_s = d_s - d_obs,s.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operators as ops


def gauss_legendre(n, K):
    """Nodes and weights of the n-point Gauss-Legendre rule on [0, K]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * K * (t + 1.0), 0.5 * K * w


def ky_rule(omega, h, nky, p, v_min):
    """Quadrature in k_y: nodes on [0, min(p omega / v_min, pi / h)] and the
    weights with the 1/pi of the inverse cosine transform."""
    K = min(p * omega / v_min, np.pi / h)
    k, w = gauss_legendre(nky, K)
    return k, w / np.pi


def assemble2d(g: ops.Grid, m, k):
    """H(k) on a grid with g.n[0] == 1: the layer-stretched 3-point rows of
    axes 1 and 2 (Kronecker sum) plus omega^2 m - k^2 on the diagonal."""
    assert g.n[0] == 1
    n1, n2 = g.n[1], g.n[2]
    mats = []
    for a, n in ((1, n1), (2, n2)):
        cp, cm = ops.axis_coeffs(g, a)
        mats.append(sp.diags([cm[1:], -(cp + cm), cp[:-1]], [-1, 0, 1], shape=(n, n), format="csr",
                             dtype=np.complex128))
    L = sp.kron(mats[0], sp.identity(n2), format="csr") + sp.kron(sp.identity(n1), mats[1], format="csr")
    diag = (g.omega ** 2) * np.asarray(m, np.float64).ravel() - k * k
    return (L + sp.diags(diag)).tocsr()


def source2d(g: ops.Grid, node, amp=1.0 + 0.0j):
    q = np.zeros(g.n, dtype=np.complex128)
    q[0, node[0], node[1]] = amp / g.h ** 2
    return q


def fields(g: ops.Grid, m, src, amp, k):
    """u~ for every source at one k_y (one LU)."""
    lu = spla.splu(assemble2d(g, m, k).tocsc())
    return [lu.solve(source2d(g, p, a).ravel()).reshape(g.n) for p, a in zip(src, amp)], lu


def misfit_gradient(g: ops.Grid, m, src, src_y, rec, rec_y, d, nky, p, v_min, amp=None, want_grad=True):
    """Data, misfit and gradient for all sources of one frequency (g.omega);
    d: [nsrc][nrec] observed (None: data only).  Returns (d_pred, f, g)."""
    src, rec = np.asarray(src), np.asarray(rec)
    amp = np.ones(len(src), np.complex128) if amp is None else np.asarray(amp)
    kq, wq = ky_rule(g.omega, g.h, nky, p, v_min)
    ns, nr = len(src), len(rec)
    dy = np.asarray(rec_y)[None, :] - np.asarray(src_y)[:, None]  # [s][r]
    d_pred = np.zeros((ns, nr), np.complex128)
    per_k = []
    for k, w in zip(kq, wq):
        us, lu = fields(g, m, src, amp, k)
        c = w * np.cos(k * dy)  # [s][r]
        for s in range(ns):
            d_pred[s] += c[s] * us[s][0, rec[:, 0], rec[:, 1]]
        per_k.append((k, c, us, lu))
    if d is None:
        return d_pred, None, None
    r = d_pred - np.asarray(d)
    f = 0.5 * float(np.sum(np.abs(r) ** 2))
    grad = np.zeros(g.n)
    if want_grad:
        for k, c, us, lu in per_k:
            for s in range(ns):
                b = np.zeros(g.n, np.complex128)
                np.add.at(b, (0, rec[:, 0], rec[:, 1]), c[s] * r[s])
                v = -lu.solve(b.ravel(), trans="H").reshape(g.n)
                grad += np.real((g.omega ** 2) * np.conj(us[s]) * v)
    return d_pred, f, grad


def misfit_gradient_pairs(g: ops.Grid, m, omegas, src, src_y, rec, rec_y, d, nky, p, v_min, amp=None, mask=None,
                          renormalise=False):
    """Sum over the selected (frequency, source) pairs; d [nfreq][nsrc][nrec]
    (None: data only).  Returns (d_pred [nfreq][nsrc][nrec], f, g)."""
    src = np.asarray(src)
    nf, ns, nr = len(omegas), len(src), len(rec)
    amp = np.ones((nf, ns), np.complex128) if amp is None else np.asarray(amp).reshape(nf, ns)
    mask = np.ones((nf, ns), bool) if mask is None else np.asarray(mask, bool).reshape(nf, ns)
    src_y = np.asarray(src_y, np.float64)
    d_pred = np.zeros((nf, ns, nr), np.complex128)
    f_tot, g_tot = 0.0, np.zeros(g.n)
    for fi, om in enumerate(omegas):
        sel = np.nonzero(mask[fi])[0]
        if len(sel) == 0:
            continue
        dd = None if d is None else np.asarray(d)[fi, sel]
        dp, f, gr = misfit_gradient(replace(g, omega=float(om)), m, src[sel], src_y[sel], rec, rec_y, dd, nky, p,
                                    v_min, amp[fi, sel])
        d_pred[fi, sel] = dp
        if d is not None:
            f_tot += f
            g_tot += gr
    npair = int(mask.sum())
    if renormalise and npair:
        f_tot /= npair
        g_tot /= npair
    return d_pred, f_tot, g_tot
