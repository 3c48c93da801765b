"""Oracle: off-grid sources and receivers by Kaiser-windowed sinc
interpolation (TEST INFRASTRUCTURE; never imported by the GPU library).

The paper discretises the delta source function, and samples fields at
receivers, with Kaiser-windowed sinc interpolation (Software Design section;
the interpolation operators Ps and Pr of the PDEfunc listing; Hicks 2002).
Definition used here, per axis, for a point at position x in node units
(node i sits at coordinate i):

    w(i) = sinc(i - x) * W(i - x),     sinc(t) = sin(pi t) / (pi t),
    W(t) = I0(b sqrt(1 - (t / r)^2)) / I0(b) for |t| <= r, else 0,

over the 2r nodes floor(x) - r + 1 .. floor(x) + r (every other node has
|i - x| > r, or sits at distance exactly r where the weight is zero for an
on-node x); nodes outside the grid are dropped (the field is zero there).
The 3D weights are the tensor product of the three axes.  r (half-width in
nodes) and b (window shape) are parameters; an on-node position gives the
Kronecker delta (sinc vanishes at the other integers), so the on-node case of
the misfit module is the special case.

  source       q = amp * sum_n w_n e_n / h^3
  receiver     (P u)_k = sum_n w_{k,n} u_n,    P^T r = sum_k w_{k,n} r_k

``fit_kaiser_b`` chooses b for a half-width r by minimising the largest
deviation from 1 of the interpolator's spectrum over wavenumbers up to kmax
(the criterion Hicks states; our own search, no table).
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from . import fwi
from . import operators as ops


def sinc(t):
    """sin(pi t) / (pi t), with sin(pi t) evaluated after reducing t to its
    nearest integer (sin(pi t) = (-1)^n sin(pi (t - n))), so that it is exactly
    zero at every nonzero integer."""
    t = np.asarray(t, dtype=np.float64)
    n = np.round(t)
    s = np.sin(np.pi * (t - n)) * np.where(np.mod(n, 2) == 0, 1.0, -1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(t == 0.0, 1.0, s / (np.pi * t))


def kaiser(t, r, b):
    t = np.asarray(t, dtype=np.float64)
    inside = np.abs(t) <= r
    arg = np.sqrt(np.clip(1.0 - (t / r) ** 2, 0.0, None))
    return np.where(inside, np.i0(b * arg) / np.i0(b), 0.0)


def weights_1d(x, n, r, b):
    """(nodes, weights) of one axis for position x (node units)."""
    base = int(np.floor(x))
    nodes = np.arange(base - r + 1, base + r + 1)
    t = nodes - x
    w = sinc(t) * kaiser(t, r, b)
    keep = (nodes >= 0) & (nodes < n)
    return nodes[keep], w[keep]


def point_weights(pos, n, r, b):
    """Flat node indices and weights of the 3D windowed sinc at pos."""
    (ix, wx), (iy, wy), (iz, wz) = (weights_1d(pos[a], n[a], r, b) for a in range(3))
    lin = ((ix[:, None, None] * n[1] + iy[None, :, None]) * n[2] + iz[None, None, :]).ravel()
    w = (wx[:, None, None] * wy[None, :, None] * wz[None, None, :]).ravel()
    return lin, w


def source(g: ops.Grid, pos, r, b, amp=1.0 + 0.0j):
    q = np.zeros(g.N, dtype=np.complex128)
    lin, w = point_weights(pos, g.n, r, b)
    q[lin] += amp * w / g.h ** 3
    return q.reshape(g.n)


def sample(u, rec_pos, r, b):
    """P u: the windowed-sinc interpolation of u at every receiver."""
    n = u.shape
    flat = u.ravel()
    out = np.zeros(len(rec_pos), dtype=np.complex128)
    for k, p in enumerate(rec_pos):
        lin, w = point_weights(p, n, r, b)
        out[k] = np.sum(w * flat[lin])
    return out


def sample_adjoint(n, rec_pos, r, b, res):
    """P^T r: every receiver's value spread back with its weights."""
    y = np.zeros(int(np.prod(n)), dtype=np.complex128)
    for k, p in enumerate(rec_pos):
        lin, w = point_weights(p, n, r, b)
        np.add.at(y, lin, w * res[k])
    return y.reshape(n)


def misfit_gradient(g: ops.Grid, m, src_pos, rec_pos, d, r, b, amp=None,
                    stencil="7pt", w27=None, solve=None):
    """f = 1/2 sum_s ||P u_s - d_s||^2 and its gradient for off-grid
    sources and receivers (one frequency), as fwi.misfit_gradient."""
    solve = solve or fwi.LUSolver(g, m, stencil, w27)
    amp = np.ones(len(src_pos), np.complex128) if amp is None else amp
    us = [solve(source(g, p, r, b, amp[s]), False) for s, p in enumerate(src_pos)]
    rs = [sample(u, rec_pos, r, b) - d[s] for s, u in enumerate(us)]
    f = 0.5 * sum(float(np.vdot(x, x).real) for x in rs)
    vs = [solve(-sample_adjoint(g.n, rec_pos, r, b, x), True) for x in rs]
    return f, fwi.gradient(g, us, vs, stencil, w27), us, vs


def misfit_gradient_pairs(g, m, omegas, src_pos, rec_pos, d, r, b, amp=None,
                          mask=None, renormalise=False, stencil="7pt", w27=None):
    """Off-grid version of fwi.misfit_gradient_pairs."""
    nf, ns = len(omegas), len(src_pos)
    amp = np.ones((nf, ns), np.complex128) if amp is None else np.asarray(amp).reshape(nf, ns)
    mask = np.ones((nf, ns), bool) if mask is None else np.asarray(mask, bool).reshape(nf, ns)
    d = np.asarray(d).reshape(nf, ns, -1)
    src_pos = np.asarray(src_pos, dtype=np.float64)
    f_tot, g_tot = 0.0, np.zeros(g.n)
    for fi, om in enumerate(omegas):
        sel = np.nonzero(mask[fi])[0]
        if len(sel) == 0:
            continue
        f, grad, _, _ = misfit_gradient(replace(g, omega=float(om)), m, src_pos[sel], rec_pos, d[fi, sel],
                                        r, b, amp=amp[fi, sel], stencil=stencil, w27=w27)
        f_tot += f
        g_tot += grad
    npair = int(mask.sum())
    if renormalise and npair > 0:
        f_tot /= npair
        g_tot /= npair
    return f_tot, g_tot


def spectral_error(r, b, kmax, nk=64, nx=32):
    """max over wavenumbers |k| <= kmax and sub-node offsets of
    |sum_n w(n - x) e^{i k (n - x)} - 1|: how far the windowed sinc is from
    an exact interpolator of band-limited signals."""
    ks = np.linspace(0.0, kmax, nk)
    worst = 0.0
    for x in np.linspace(0.0, 1.0, nx, endpoint=False):
        nodes = np.arange(-r + 1, r + 1)
        t = nodes - x
        w = sinc(t) * kaiser(t, r, b)
        resp = np.exp(1j * np.outer(ks, t)) @ w
        worst = max(worst, float(np.abs(resp - 1.0).max()))
    return worst


def fit_kaiser_b(r, kmax, lo=0.0, hi=20.0, iters=80):
    """b minimising spectral_error(r, b, kmax) (golden-section search; the
    error is unimodal in b over this bracket for the half-widths used)."""
    gr = (np.sqrt(5.0) - 1.0) / 2.0
    a, c = lo, hi
    x1, x2 = c - gr * (c - a), a + gr * (c - a)
    f1, f2 = spectral_error(r, x1, kmax), spectral_error(r, x2, kmax)
    for _ in range(iters):
        if f1 < f2:
            c, x2, f2 = x2, x1, f1
            x1 = c - gr * (c - a)
            f1 = spectral_error(r, x1, kmax)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + gr * (c - a)
            f2 = spectral_error(r, x2, kmax)
    return 0.5 * (a + c)
