"""Oracle: discrete 3D Helmholtz operators in complex128 (TEST INFRASTRUCTURE).

Only tests, the smoke check and the bench's CPU-baseline leg use this module;
the GPU library never imports it and shares no code with it.

What is defined here (paper, Preamble and Appendix A)
------------------------------------------------------
The problem is the constant-density Helmholtz equation in the form
``L u + omega^2 A diag(m) u = q`` (Appendix A, the linear system preceding
eq. dH), with ``m = 1/v^2`` (slowness squared) on the layer-extended grid,
zero Dirichlet data outside the grid (Preamble: rectangular domain with zero
Dirichlet conditions) and a perfectly matched layer in which each derivative
is replaced by ``(1/eta) d/dx`` (Preamble, extended-domain equation).

* Grid: nodes ``p = (i, j, k)`` with ``0 <= i < nx`` etc., C order, z
  fastest.  Values outside the grid are zero.
* Layer profile (the paper leaves eta open): per axis, with t the node
  coordinate in *fine-grid* units, ``d(t) = max(0, npml - t, t - (n-1-npml))``,
  ``sigma(t) = sigma_max (d/npml)^2``,
  ``sigma_max = 3 v_ref ln(1/R) / (2 npml h)``, and the stretch
  ``s(t) = 1 + i sigma(t)/omega`` (decays the outgoing ``exp(+i kappa r)``
  wave that the Sommerfeld condition of eq. helmholtz selects).
* 7-point operator, per axis a and node p (difference form):
  ``(L7 u)_p = sum_a [cp_a (u_{p+e_a} - u_p) - cm_a (u_p - u_{p-e_a})]``,
  ``cp = 1/(h^2 s(p) s(p+1/2))``, ``cm = 1/(h^2 s(p) s(p-1/2))``,
  i.e. ``(1/s) d/dx ((1/s) du/dx)`` with half-node stretches.
  ``H7 = L7 + omega^2 diag(m)`` (A = I).
* Compact 27-point operator (the 3D kernel the paper uses, Software Design,
  SPOT-operator paragraph): on rows whose 26 neighbours all lie outside the
  layer, ``L27 = w1 L1 + w2 L2 + w3 L3`` with the axis, face-diagonal and
  body-diagonal second-difference Laplacians; elsewhere the 7-point layer row.
  The mass matrix A distributes ``m*u`` with weights (wm1 centre, wm2 faces,
  wm3 edges, wm4 corners) on every row, so A is real symmetric.
* Adjoint ``H^H`` is the conjugate transpose, written out row by row.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from itertools import product

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# grid and absorbing layer
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Grid:
    """One level of the computational grid.

    n       nodes per axis on this level
    h       spacing on this level
    npml    layer width in fine-grid nodes
    n_fine  fine-grid node counts (the layer profile is defined on them)
    stride  fine nodes per node of this level (2**level)
    omega   angular frequency
    v_ref   reference velocity of the layer profile
    R       nominal layer reflection coefficient
    """

    n: tuple
    h: float
    npml: int
    omega: float
    v_ref: float
    R: float = 1e-3
    n_fine: tuple = None
    stride: int = 1

    def __post_init__(self):
        if self.n_fine is None:
            object.__setattr__(self, "n_fine", tuple(self.n))

    @property
    def N(self):
        return int(np.prod(self.n))

    @property
    def h_fine(self):
        return self.h / self.stride


def make_grid(n, h, npml, omega, v_ref, R=1e-3):
    return Grid(n=tuple(int(a) for a in n), h=float(h), npml=int(npml),
                omega=float(omega), v_ref=float(v_ref), R=float(R))


def coarsen(g: Grid) -> Grid:
    """Next coarser level: n_c = floor(n/2) + 1 nodes, coarse node I at fine
    coordinate 2I, spacing 2h, same frequency and layer profile."""
    return replace(g, n=tuple(a // 2 + 1 for a in g.n), h=2.0 * g.h,
                   stride=2 * g.stride)


def sigma_max(g: Grid) -> float:
    if g.npml == 0:
        return 0.0
    return 3.0 * g.v_ref * np.log(1.0 / g.R) / (2.0 * g.npml * g.h_fine)


def layer_sigma(g: Grid, axis: int, t) -> np.ndarray:
    """Damping sigma at level coordinate t (integer = node, +-1/2 = half node)."""
    tf = np.asarray(t, dtype=np.float64) * g.stride
    if g.npml == 0:
        return np.zeros_like(tf)
    nf = g.n_fine[axis]
    d = np.maximum(0.0, np.maximum(g.npml - tf, tf - (nf - 1 - g.npml)))
    return sigma_max(g) * (d / g.npml) ** 2


def stretch(g: Grid, axis: int, t) -> np.ndarray:
    """Complex coordinate stretch s(t) = 1 + i sigma(t)/omega."""
    return 1.0 + 1j * layer_sigma(g, axis, t) / g.omega


def coeffs_from_stretch(h, s_node, s_plus, s_minus):
    """1D coefficients of (1/s) d/dx (1/s) d/dx at the nodes of one axis."""
    cp = 1.0 / (h * h * s_node * s_plus)
    cm = 1.0 / (h * h * s_node * s_minus)
    return cp, cm


def axis_coeffs(g: Grid, axis: int):
    """(cp, cm), complex arrays of length n[axis], for the 7-point layer row."""
    i = np.arange(g.n[axis], dtype=np.float64)
    return coeffs_from_stretch(g.h, stretch(g, axis, i),
                               stretch(g, axis, i + 0.5),
                               stretch(g, axis, i - 0.5))


# ----------------------------------------------------------------------------
# helpers: zero-padded shifts
# ----------------------------------------------------------------------------

def shift(x: np.ndarray, d) -> np.ndarray:
    """Return y with y[p] = x[p + d] (zero where p + d is outside the grid)."""
    y = np.zeros_like(x)
    src, dst = [], []
    for a, da in enumerate(d):
        n = x.shape[a]
        if da >= 0:
            src.append(slice(da, n))
            dst.append(slice(0, n - da))
        else:
            src.append(slice(0, n + da))
            dst.append(slice(-da, n))
    y[tuple(dst)] = x[tuple(src)]
    return y


def _bcast(v, axis):
    s = [1, 1, 1]
    s[axis] = v.size
    return v.reshape(s)


# ----------------------------------------------------------------------------
# 7-point operator
# ----------------------------------------------------------------------------

def laplacian7(g: Grid, x: np.ndarray, adjoint: bool = False, coeffs=None):
    """Layer-stretched 7-point Laplacian L7 (or its conjugate transpose).

    Forward row p: sum_a cp_a(p)(x_{p+e_a} - x_p) - cm_a(p)(x_p - x_{p-e_a}).
    Adjoint row p gathers the conjugated column p of L7:
    conj(L7[p+e_a, p]) = conj(cm_a(p+1)),  conj(L7[p-e_a, p]) = conj(cp_a(p-1)),
    conj(L7[p, p]) = -conj(cp_a(p) + cm_a(p)).
    ``coeffs`` optionally overrides the per-axis (cp, cm) pairs.
    """
    x = np.asarray(x, dtype=np.complex128)
    y = np.zeros_like(x)
    for a in range(3):
        cp, cm = coeffs[a] if coeffs is not None else axis_coeffs(g, a)
        e = [0, 0, 0]
        e[a] = 1
        xp = shift(x, e)
        xm = shift(x, [-v for v in e])
        if not adjoint:
            y += _bcast(cp, a) * (xp - x) - _bcast(cm, a) * (x - xm)
        else:
            # coefficients of the rows p+e_a and p-e_a (zero-extended)
            cm_next = np.concatenate([cm[1:], [0.0]])
            cp_prev = np.concatenate([[0.0], cp[:-1]])
            y += (_bcast(np.conj(cm_next), a) * xp
                  + _bcast(np.conj(cp_prev), a) * xm
                  - _bcast(np.conj(cp + cm), a) * x)
    return y


def apply7(g: Grid, m: np.ndarray, x: np.ndarray, adjoint: bool = False):
    """H7 x = L7 x + omega^2 m x   (or H7^H x = L7^H x + omega^2 m x)."""
    x = np.asarray(x, dtype=np.complex128)
    return laplacian7(g, x, adjoint) + (g.omega ** 2) * np.asarray(m) * x


def assemble7(g: Grid, m: np.ndarray) -> sp.csr_matrix:
    """Independent construction of H7 as a sparse matrix from 1D factors:
    H7 = sum_a I (x) (D_a^-1 K_a) (x) I + omega^2 diag(m), where the 1D
    factor is the tridiagonal matrix of (1/s) d/dx (1/s) d/dx."""
    mats = []
    for a in range(3):
        cp, cm = axis_coeffs(g, a)
        n = g.n[a]
        B = sp.diags([cm[1:], -(cp + cm), cp[:-1]], [-1, 0, 1],
                     shape=(n, n), format="csr", dtype=np.complex128)
        eyes = [sp.identity(g.n[b], format="csr") for b in range(3)]
        eyes[a] = B
        mats.append(sp.kron(sp.kron(eyes[0], eyes[1]), eyes[2], format="csr"))
    H = mats[0] + mats[1] + mats[2]
    H = H + sp.diags((g.omega ** 2) * np.asarray(m, np.float64).ravel())
    return H.tocsr()


# ----------------------------------------------------------------------------
# compact 27-point operator
# ----------------------------------------------------------------------------

def offsets27():
    return [d for d in product((-1, 0, 1), repeat=3)]


def offset_class(d) -> int:
    """0 centre, 1 face (6), 2 edge (12), 3 corner (8)."""
    return int(sum(abs(v) for v in d))


def laplacian27_weights(w27, h):
    """Per-class weights of L27 = w1 L1 + w2 L2 + w3 L3.

    L1 = h^-2 sum over 3 axes of the second difference;
    L2 = L1/3 + (1/(6 h^2)) sum over the 6 face diagonals;
    L3 = (1/(4 h^2)) sum over the 4 body diagonals;
    second difference along d: u(p+d) + u(p-d) - 2u(p).
    Returns (centre, face, edge, corner).
    """
    w1, w2, w3 = w27[0], w27[1], w27[2]
    h2 = h * h
    # per-class coefficients of L1, L2, L3
    L1 = (-6.0, 1.0, 0.0, 0.0)
    L2 = (-6.0 / 3.0 - 12.0 / 6.0, 1.0 / 3.0, 1.0 / 6.0, 0.0)
    L3 = (-8.0 / 4.0, 0.0, 0.0, 1.0 / 4.0)
    return tuple((w1 * L1[c] + w2 * L2[c] + w3 * L3[c]) / h2 for c in range(4))


def mass27_weights(w27):
    return (w27[3], w27[4], w27[5], w27[6])


def stencil27(x: np.ndarray, class_w) -> np.ndarray:
    """sum_d class_w[class(d)] x_{p+d} over the 27 offsets (zero outside)."""
    y = np.zeros_like(x)
    for d in offsets27():
        c = class_w[offset_class(d)]
        if c != 0.0:
            y += c * shift(x, d)
    return y


def interior27_mask(g: Grid) -> np.ndarray:
    """True on rows whose node and 26 neighbours all lie where sigma == 0."""
    masks = []
    for a in range(3):
        i = np.arange(g.n[a], dtype=np.float64)
        ok = (layer_sigma(g, a, i - 1) == 0.0) & (layer_sigma(g, a, i + 1) == 0.0)
        masks.append(ok)
    return (masks[0][:, None, None] & masks[1][None, :, None]
            & masks[2][None, None, :])


def apply27(g: Grid, m: np.ndarray, x: np.ndarray, w27, adjoint=False):
    """Compact 27-point Helmholtz operator or its conjugate transpose.

    H27 = Mi L27 + (I - Mi) L7 + omega^2 A diag(m), Mi = diag(interior mask).
    L27 and A are real symmetric, so
    H27^H = L27 Mi + L7^H (I - Mi) + omega^2 diag(m) A.
    """
    x = np.asarray(x, dtype=np.complex128)
    mask = interior27_mask(g)
    lw = laplacian27_weights(w27, g.h)
    aw = mass27_weights(w27)
    w2 = g.omega ** 2
    m = np.asarray(m, dtype=np.float64)
    if not adjoint:
        lap = np.where(mask, stencil27(x, lw), laplacian7(g, x))
        return lap + w2 * stencil27(m * x, aw)
    lap = stencil27(np.where(mask, x, 0.0), lw) + \
        laplacian7(g, np.where(mask, 0.0, x), adjoint=True)
    return lap + w2 * m * stencil27(x, aw)


def assemble27(g: Grid, m: np.ndarray, w27) -> sp.csr_matrix:
    """Sparse H27 built entry by entry from the row definitions (COO)."""
    n = g.n
    N = g.N
    idx = np.arange(N).reshape(n)
    mask = interior27_mask(g).ravel()
    lw = laplacian27_weights(w27, g.h)
    aw = mass27_weights(w27)
    w2 = g.omega ** 2
    mflat = np.asarray(m, np.float64).ravel()
    rows, cols, vals = [], [], []
    P = np.stack(np.meshgrid(*[np.arange(a) for a in n], indexing="ij"),
                 axis=-1).reshape(-1, 3)
    for d in offsets27():
        Q = P + np.array(d)
        ok = np.all((Q >= 0) & (Q < np.array(n)), axis=1)
        r = np.nonzero(ok)[0]
        c = idx[Q[ok, 0], Q[ok, 1], Q[ok, 2]]
        cl = offset_class(d)
        # interior Laplacian rows
        sel = mask[r]
        if lw[cl] != 0.0:
            rows.append(r[sel]); cols.append(c[sel])
            vals.append(np.full(sel.sum(), lw[cl], np.complex128))
        # mass term on all rows: omega^2 * aw * m_col
        if aw[cl] != 0.0:
            rows.append(r); cols.append(c)
            vals.append((w2 * aw[cl] * mflat[c]).astype(np.complex128))
    # layer rows: 7-point stretched Laplacian
    L7 = assemble7(g, np.zeros(n)).tocoo()
    keep = ~mask[L7.row]
    rows.append(L7.row[keep]); cols.append(L7.col[keep]); vals.append(L7.data[keep])
    H = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    H.sum_duplicates()
    return H


def apply(g: Grid, m, x, adjoint=False, stencil="7pt", w27=None):
    """Dispatch on the stencil name."""
    if stencil == "7pt":
        return apply7(g, m, x, adjoint)
    return apply27(g, m, x, w27, adjoint)


def assemble(g: Grid, m, stencil="7pt", w27=None):
    if stencil == "7pt":
        return assemble7(g, m)
    return assemble27(g, m, w27)


# ----------------------------------------------------------------------------
# closed forms used by the pins
# ----------------------------------------------------------------------------

def symbol27(kvec, h, w27, omega2m):
    """Plane-wave symbol of the interior 27-point row for exp(i k.x):
    H u = symbol * u with symbol = sum_d w(d) exp(i k.d h) (Laplacian part)
    + omega^2 m * sum_d wm(d) exp(i k.d h) (mass part), as cosine sums."""
    c = [np.cos(ka * h) for ka in kvec]
    lw = laplacian27_weights(w27, h)
    aw = mass27_weights(w27)
    s1 = c[0] + c[1] + c[2]
    s2 = c[0] * c[1] + c[0] * c[2] + c[1] * c[2]
    s3 = c[0] * c[1] * c[2]
    lap = lw[0] + 2 * lw[1] * s1 + 4 * lw[2] * s2 + 8 * lw[3] * s3
    mass = aw[0] + 2 * aw[1] * s1 + 4 * aw[2] * s2 + 8 * aw[3] * s3
    return lap + omega2m * mass
