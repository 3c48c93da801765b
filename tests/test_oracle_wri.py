"""Pins of the WRI (penalty method) oracle: the field against a dense
least-squares solve of the stacked system [P_r; lambda H] u = [d; lambda q]
by SVD (a different algorithm from the normal equations), the optimality of
the field (phi below the reduced misfit, gradient in u zero), the limit
lambda -> infinity (misfit and gradient of the reduced formulation, error
O(1/lambda^2)), and the gradient against central differences of the
objective re-solved from scratch (7-point and 27-point)."""
from dataclasses import replace

import numpy as np

from oracle import fwi, wri
from oracle import operators as ops
import workloads


def _case(seed=120, n=(9, 8, 8), npml=2, stencil="7pt"):
    w = workloads.layered_random_workload(n, 25.0, npml, 6.0, nsrc_xy=(2, 1), nrec_xy=(3, 3), seed=seed)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    rng = np.random.default_rng(seed)
    solve = fwi.LUSolver(g, w.m * (1 + 0.05 * rng.standard_normal(w.m.shape)))
    d = np.stack([fwi.sample(solve(fwi.point_source(g, p)), w.rec) for p in w.src])
    H = ops.assemble(g, w.m, stencil, workloads.W27_DEFAULT if stencil == "27pt" else None)
    lam = 1.0 / spla_norm_est(H)  # lambda^2 H^H H and P^T P of comparable size
    return w, g, d, lam


def spla_norm_est(H):
    """Largest singular value of H by dense SVD (tiny grids only)."""
    return float(np.linalg.svd(H.toarray(), compute_uv=False)[0])


def test_field_equals_dense_stacked_least_squares():
    for stencil in ("7pt", "27pt"):
        w27 = workloads.W27_DEFAULT if stencil == "27pt" else None
        w, g, d, lam = _case(stencil=stencil)
        us, qs, H, P = wri.wri_fields(g, w.m, w.src, w.rec, d, lam, stencil=stencil, w27=w27)
        Hd, Pd = H.toarray(), P.toarray()
        for s in range(len(w.src)):
            A = np.vstack([Pd, lam * Hd])
            b = np.concatenate([d[s], lam * qs[s].ravel()])
            x = np.linalg.lstsq(A, b, rcond=None)[0]
            assert np.linalg.norm(x - us[s].ravel()) <= 1e-9 * np.linalg.norm(x)


def test_field_is_optimal():
    """phi(m, u(m)) <= phi(m, H^{-1} q) = the reduced misfit, and the
    gradient of phi in u vanishes at u(m)."""
    w, g, d, lam = _case(seed=121)
    f, _, us = wri.wri_misfit_gradient(g, w.m, w.src, w.rec, d, lam)
    f_red = fwi.misfit_gradient(g, w.m, w.src, w.rec, d)[0]
    assert f < f_red
    _, qs, H, P = wri.wri_fields(g, w.m, w.src, w.rec, d, lam)
    for s, u in enumerate(us):
        gu = P.T @ (P @ u.ravel() - d[s]) + lam ** 2 * (H.conj().T @ (H @ u.ravel() - qs[s].ravel()))
        assert np.linalg.norm(gu) <= 1e-9 * np.linalg.norm(P.T @ d[s])


def test_large_lambda_limit_is_the_reduced_objective():
    """As lambda grows, f and grad f tend to the reduced misfit and its
    adjoint-state gradient, with error O(1/lambda^2) (ratio 4 per doubling)."""
    w, g, d, lam = _case(seed=122)
    f0, g0, _, _ = fwi.misfit_gradient(g, w.m, w.src, w.rec, d)
    errs = []
    for k in (1.0, 2.0):
        L = 1e3 * k * lam
        f, gr, _ = wri.wri_misfit_gradient(g, w.m, w.src, w.rec, d, L)
        errs.append((abs(f - f0) / f0, np.linalg.norm(gr - g0) / np.linalg.norm(g0)))
    assert errs[0][0] < 5e-3 and errs[0][1] < 5e-3  # (lambda much larger: lambda^2 (H u - q) loses digits)
    assert 3.5 < errs[0][0] / errs[1][0] < 4.5
    assert 3.5 < errs[0][1] / errs[1][1] < 4.5


def test_gradient_by_resolving():
    """grad f = lambda^2 T^*(H u - q) against (f(m + e) - f(m - e)) / 2e with
    u(m +- e) re-solved, two frequencies, masked pairs, 1/#pairs."""
    rng = np.random.default_rng(123)
    for stencil in ("7pt", "27pt"):
        w27 = workloads.W27_DEFAULT if stencil == "27pt" else None
        w, g, d1, lam = _case(seed=123, stencil=stencil)
        omegas = [2 * np.pi * 5.0, 2 * np.pi * 6.0]
        d = np.stack([d1, 1.1 * d1])
        mask = np.array([[True, True], [True, False]])
        amp = np.array([[1.0, 0.5 - 0.2j], [1.2j, 1.0]])
        f, grad, _ = wri.wri_misfit_gradient_pairs(g, w.m, omegas, w.src, w.rec, d, lam, amp=amp, mask=mask,
                                                   renormalise=True, stencil=stencil, w27=w27)
        lo, hi = g.npml, np.array(g.n) - g.npml
        for _ in range(4):
            k = tuple(rng.integers(lo, hi[a]) for a in range(3))
            eps = 1e-5 * w.m[k]
            mp, mm = w.m.copy(), w.m.copy()
            mp[k] += eps
            mm[k] -= eps
            fp = wri.wri_misfit_gradient_pairs(g, mp, omegas, w.src, w.rec, d, lam, amp=amp, mask=mask,
                                               renormalise=True, stencil=stencil, w27=w27)[0]
            fm = wri.wri_misfit_gradient_pairs(g, mm, omegas, w.src, w.rec, d, lam, amp=amp, mask=mask,
                                               renormalise=True, stencil=stencil, w27=w27)[0]
            fd = (fp - fm) / (2 * eps)
            assert abs(grad[k] - fd) <= 1e-6 * np.abs(grad).max(), (stencil, k, grad[k], fd)
