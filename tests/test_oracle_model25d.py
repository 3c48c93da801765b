"""Pins of the 2.5D oracle: the Gauss-Legendre rule's exactness on
polynomials, the 2D operator's Dirichlet eigenvalues and adjoint, the 2D
field of one k_y against the closed-form 2D Green's functions (oscillating
below omega/v, decaying above: the sign of the k_y^2 term), the 2.5D sum
against the 3D Green's function of a constant medium (the paper's own check
of the method), and the gradient against central differences of the
re-solved objective."""
from dataclasses import replace

import numpy as np
import scipy.sparse.linalg as spla
from scipy import special

from oracle import model25d as m25
from oracle import operators as ops


def test_gauss_legendre_exact_on_polynomials():
    K = 0.37
    for n in (3, 8, 20):
        k, w = m25.gauss_legendre(n, K)
        assert np.all((k > 0) & (k < K)) and np.all(w > 0)
        for j in range(2 * n):
            assert abs(np.sum(w * k ** j) - K ** (j + 1) / (j + 1)) <= 1e-12 * K ** (j + 1)
    # the k_y rule: cut at min(p omega / v_min, pi / h), 1/pi folded in
    k, w = m25.ky_rule(2 * np.pi * 5.0, 10.0, 16, 2.0, 2000.0)
    assert abs(w.sum() * np.pi - 2.0 * 2 * np.pi * 5.0 / 2000.0) <= 1e-12
    k, w = m25.ky_rule(2 * np.pi * 5.0, 100.0, 16, 50.0, 2000.0)
    assert abs(w.sum() * np.pi - np.pi / 100.0) <= 1e-12


def test_operator_dirichlet_eigenvalues_and_adjoint():
    """No layer, constant m, k: the sine modes are eigenvectors with
    eigenvalue omega^2 m - k^2 - sum_a (4/h^2) sin^2(pi l_a / (2 (n_a + 1)))."""
    n1, n2, h, om, k = 14, 11, 7.0, 2.0, 0.05
    g = ops.make_grid((1, n1, n2), h, 0, om, 1500.0)
    m = np.full(g.n, 3e-7)
    H = m25.assemble2d(g, m, k)
    J, K = np.meshgrid(np.arange(1, n1 + 1), np.arange(1, n2 + 1), indexing="ij")
    for l1, l2 in ((1, 1), (3, 5), (n1, n2)):
        u = np.sin(np.pi * l1 * J / (n1 + 1)) * np.sin(np.pi * l2 * K / (n2 + 1))
        lam = om ** 2 * 3e-7 - k * k - 4 / h ** 2 * (np.sin(np.pi * l1 / (2 * (n1 + 1))) ** 2 +
                                                   np.sin(np.pi * l2 / (2 * (n2 + 1))) ** 2)
        assert np.linalg.norm(H @ u.ravel() - lam * u.ravel()) <= 1e-12 * abs(lam) * np.linalg.norm(u)
    g = ops.make_grid((1, n1, n2), h, 3, om, 1500.0)
    H = m25.assemble2d(g, m, k)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(g.N) + 1j * rng.standard_normal(g.N)
    y = rng.standard_normal(g.N) + 1j * rng.standard_normal(g.N)
    assert abs(np.vdot(y, H @ x) - np.vdot(H.conj().T @ y, x)) <= 1e-12 * np.linalg.norm(H @ x) * np.linalg.norm(y)


def _constant_case():
    n, h, npml, f, v = 121, 10.0, 20, 5.0, 2000.0
    om = 2 * np.pi * f
    g = ops.make_grid((1, n, n), h, npml, om, v)
    m = np.full(g.n, 1.0 / v ** 2)
    J, K = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r2 = h * np.hypot(J - 60, K - 60)
    sel = np.argwhere((r2 >= 150) & (r2 <= 350))
    sel = sel[np.random.default_rng(0).choice(len(sel), 60, replace=False)]
    return g, m, om / v, sel, r2[sel[:, 0], sel[:, 1]]


def test_single_ky_field_is_the_2d_greens_function():
    """(d_xx + d_zz + kappa^2 - k^2) u = delta: -(i/4) H0(sqrt(kappa^2 - k^2) r)
    for k < kappa, -K0(sqrt(k^2 - kappa^2) r) / (2 pi) for k > kappa."""
    g, m, kap, rec, r = _constant_case()
    for k in (0.0, 0.6 * kap, 1.5 * kap):
        lu = spla.splu(m25.assemble2d(g, m, k).tocsc())
        u = lu.solve(m25.source2d(g, (60, 60)).ravel()).reshape(g.n)[0, rec[:, 0], rec[:, 1]]
        if k < kap:
            ref = -0.25j * special.hankel1(0, np.sqrt(kap ** 2 - k ** 2) * r)
        else:
            ref = -special.k0(np.sqrt(k ** 2 - kap ** 2) * r) / (2 * np.pi)
        assert np.linalg.norm(u - ref) <= 0.02 * np.linalg.norm(ref), k / kap


def test_25d_sum_is_the_3d_greens_function():
    """Constant medium: the quadrature of the 2D fields over k_y gives
    -exp(i kappa R) / (4 pi R) at receivers off the source's line, R the 3D
    distance (200 nodes on [0, 4 kappa]: within 2 % over the receivers at
    offsets 0, 100 and 200 m along the invariant axis)."""
    g, m, kap, rec, r = _constant_case()
    recs = np.concatenate([rec, rec, rec])
    y = np.concatenate([np.zeros(len(rec)), np.full(len(rec), 100.0), np.full(len(rec), 200.0)])
    # the source at y_s = 50 m, the receivers 0, 100, 200 m beyond it along y
    dp, _, _ = m25.misfit_gradient(g, m, [(60, 60)], [50.0], recs, y + 50.0, None, 200, 4.0, 2000.0)
    R = np.sqrt(np.concatenate([r, r, r]) ** 2 + y ** 2)
    ref = -np.exp(1j * kap * R) / (4 * np.pi * R)
    for s in range(3):
        part = slice(s * len(rec), (s + 1) * len(rec))
        assert np.linalg.norm(dp[0][part] - ref[part]) <= 0.02 * np.linalg.norm(ref[part])


def test_gradient_by_resolving():
    """Two frequencies, three sources with their own y, a mask, amplitudes
    and 1/#pairs: g against (f(m + e) - f(m - e)) / 2e, the quadrature fixed
    by (p, v_min)."""
    rng = np.random.default_rng(11)
    n1, n2, h, npml = 26, 22, 20.0, 4
    g = ops.make_grid((1, n1, n2), h, npml, 1.0, 3000.0)
    v = 1800.0 + 600.0 * rng.random(g.n)
    m = 1.0 / v ** 2
    omegas = [2 * np.pi * 5.0, 2 * np.pi * 6.0]
    src = np.array([(8, 5), (13, 6), (18, 5)])
    src_y = np.array([0.0, 40.0, -30.0])
    rec = np.array([(j, 17) for j in range(5, 21, 2)])
    rec_y = np.linspace(-100.0, 120.0, len(rec))
    mask = np.array([[True, False, True], [True, True, True]])
    amp = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    d = (rng.standard_normal((2, 3, len(rec))) + 1j * rng.standard_normal((2, 3, len(rec)))) * 1e-4
    args = (omegas, src, src_y, rec, rec_y, d, 10, 1.5, 1800.0)
    _, f, grad = m25.misfit_gradient_pairs(g, m, *args, amp=amp, mask=mask, renormalise=True)
    for _ in range(4):
        k = (0, int(rng.integers(npml, n1 - npml)), int(rng.integers(npml, n2 - npml)))
        eps = 1e-4 * m[k]
        mp, mm = m.copy(), m.copy()
        mp[k] += eps
        mm[k] -= eps
        fp = m25.misfit_gradient_pairs(g, mp, *args, amp=amp, mask=mask, renormalise=True)[1]
        fm = m25.misfit_gradient_pairs(g, mm, *args, amp=amp, mask=mask, renormalise=True)[1]
        assert abs(grad[k] - (fp - fm) / (2 * eps)) <= 1e-6 * np.abs(grad).max()
