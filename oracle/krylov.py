"""Oracle: restarted GMRES(k) and flexible GMRES(k) in complex128
(TEST INFRASTRUCTURE; never imported by the GPU library).

Both follow the textbook methods the paper builds on (ML-GMRES section:
GMRES smoothers with an identity preconditioner, FGMRES for the outer and
coarse solves because the preconditioner changes from one iteration to the
next): Arnoldi with modified Gram-Schmidt, Givens rotations on the upper
Hessenberg matrix, the small least-squares problem solved by back
substitution, restart after ``k`` inner steps.

Conventions (the paper leaves them open): relative residual
``||b - A x||_2 / ||b||_2``; the Krylov dimension per restart cycle is ``k``
("inner" iterations) and ``cycles`` is the number of restarts ("outer"
iterations), the reading of GMRES(k_o, k_i) that matches the paper's storage
counts of k_i+5 and 2 k_i+6 vectors.  With ``tol=None`` the method runs a
fixed number of cycles with no stopping test (the smoother mode).
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    """<a, b> = a^H b (conjugate-linear in the first argument)."""
    return np.vdot(a, b)


def _givens(a, b):
    """Complex Givens rotation (c real, s complex) with
    [c, s; -conj(s), c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b)
    t = abs(a)
    nrm = np.hypot(abs(a), abs(b))
    c = t / nrm
    s = (a / t) * np.conj(b) / nrm
    r = (a / t) * nrm
    return c, s, r


def _arnoldi_cycle(A, r0, beta, k, M=None):
    """One Arnoldi cycle of length <= k from residual r0 (norm beta).

    Returns (basis V, preconditioned directions Z or None, y, residual
    estimate, number of steps).  Hessenberg columns are reduced with Givens
    rotations as they are produced; a zero subdiagonal (happy breakdown)
    ends the cycle early.
    """
    V = [r0 / beta]
    Z = [] if M is not None else None
    Hm = np.zeros((k + 1, k), dtype=np.complex128)
    cs = np.zeros(k)
    sn = np.zeros(k, dtype=np.complex128)
    g = np.zeros(k + 1, dtype=np.complex128)
    g[0] = beta
    j_done = 0
    for j in range(k):
        if M is not None:
            z = M(V[j])
            Z.append(z)
            w = A(z)
        else:
            w = A(V[j])
        # modified Gram-Schmidt
        for i in range(j + 1):
            Hm[i, j] = _dot(V[i], w)
            w = w - Hm[i, j] * V[i]
        Hm[j + 1, j] = np.linalg.norm(w)
        # apply previous rotations to column j
        for i in range(j):
            a, b = Hm[i, j], Hm[i + 1, j]
            Hm[i, j] = cs[i] * a + sn[i] * b
            Hm[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * b
        c, s, r = _givens(Hm[j, j], Hm[j + 1, j])
        cs[j], sn[j] = c, s
        Hm[j, j] = r
        Hm[j + 1, j] = 0.0
        g[j + 1] = -np.conj(s) * g[j]
        g[j] = c * g[j]
        j_done = j + 1
        hnext = abs(np.linalg.norm(w))
        if hnext == 0.0:
            break
        V.append(w / hnext)
    # back substitution R y = g
    R = Hm[:j_done, :j_done]
    y = np.zeros(j_done, dtype=np.complex128)
    for i in range(j_done - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:j_done] @ y[i + 1:j_done]) / R[i, i]
    return V, Z, y, abs(g[j_done]), j_done


def gmres(A, b, x0=None, k=20, cycles=1, tol=None, M=None, flexible=False,
          history=None):
    """Restarted (F)GMRES(k) for A x = b.

    A        callable x -> A x
    M        optional right preconditioner (callable); with ``flexible`` the
             directions z_j = M(v_j) are stored and x = x0 + Z y (FGMRES),
             otherwise x = x0 + M(V y) (right-preconditioned GMRES)
    cycles   maximum number of restart cycles
    tol      relative residual target; None = run all cycles (smoother)
    history  optional list receiving the true relative residual per cycle

    Returns (x, info) with info = dict(cycles, steps, relres).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    steps = 0
    done = 0
    relres = np.inf
    if bnorm == 0.0:
        return np.zeros_like(b), dict(cycles=0, steps=0, relres=0.0)
    for cyc in range(cycles):
        r = b - A(x)
        beta = np.linalg.norm(r)
        relres = beta / bnorm
        if history is not None:
            history.append(relres)
        if tol is not None and relres <= tol:
            break
        if beta == 0.0:
            break
        if flexible:
            V, Z, y, _, nj = _arnoldi_cycle(A, r, beta, k, M)
        elif M is not None:
            V, Z, y, _, nj = _arnoldi_cycle(lambda v: A(M(v)), r, beta, k)
        else:
            V, Z, y, _, nj = _arnoldi_cycle(A, r, beta, k)
        steps += nj
        done = cyc + 1
        if flexible:
            for j in range(nj):
                x = x + y[j] * Z[j]
        else:
            upd = np.zeros_like(b)
            for j in range(nj):
                upd = upd + y[j] * V[j]
            x = x + (M(upd) if M is not None else upd)
    else:
        relres = np.linalg.norm(b - A(x)) / bnorm
        if history is not None:
            history.append(relres)
    return x, dict(cycles=done, steps=steps, relres=float(relres))


def fgmres(A, b, M, x0=None, k=5, cycles=1, tol=None, history=None):
    """Flexible GMRES(k): variable right preconditioner M, x = x0 + Z_k y."""
    return gmres(A, b, x0=x0, k=k, cycles=cycles, tol=tol, M=M,
                 flexible=True, history=history)


def arnoldi_relation(A, v0, k):
    """Return (V_{k+1}, Hbar_k) from k MGS-Arnoldi steps (no rotations), for
    the pin A V_k = V_{k+1} Hbar_k and V^H V = I."""
    V = [v0 / np.linalg.norm(v0)]
    H = np.zeros((k + 1, k), dtype=np.complex128)
    for j in range(k):
        w = A(V[j])
        for i in range(j + 1):
            H[i, j] = _dot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j])
    return np.stack(V, axis=1), H
