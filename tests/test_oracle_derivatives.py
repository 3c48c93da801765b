"""Pins of the derivative oracle (Jacobian, its adjoint, Gauss-Newton and full
Hessian products; Table derivstuff, Appendix A) against things other than
itself: central differences of the forward map and of the gradient computed by
re-solving from scratch, the paper's Taylor test, a dense Jacobian built
column by column from finite differences, the adjoint identities of the
paper's adjoint-test table, and the zero-residual special case (full Hessian =
Gauss-Newton Hessian)."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import derivatives as dv
from oracle import fwi
from oracle import operators as ops
import workloads

W27 = (0.55, 0.3, 0.15, 0.0, 0.06, 0.0025, -0.001)


def _w27_valid(w):
    w = list(w)
    w[3] = 1.0 - 6 * w[4] - 12 * w[5] - 8 * w[6]
    w[0] = 1.0 - w[1] - w[2]
    return tuple(w)


STENCILS = (("7pt", None), ("27pt", _w27_valid(W27)))


def _case(seed=40, n=(13, 12, 11), npml=3, nsrc=(2, 1), nrec=(4, 3)):
    w = workloads.layered_random_workload(n, 25.0, npml, 6.0, nsrc_xy=nsrc,
                                          nrec_xy=nrec, seed=seed)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    rng = np.random.default_rng(seed)
    d = (rng.standard_normal((len(w.src), len(w.rec)))
         + 1j * rng.standard_normal((len(w.src), len(w.rec)))) * 1e-4
    # a smooth model perturbation (relative size ~ 1)
    dm = workloads.gaussian_random_field(rng, g.n, 2.0) * w.m
    return w, g, d, dm, rng


@pytest.mark.parametrize("stencil,w27", STENCILS)
def test_jacobian_matches_central_difference_of_forward_map(stencil, w27):
    """J dm vs (F(m + e dm) - F(m - e dm)) / 2e with every field re-solved by
    sparse LU: agreement to the O(e^2) truncation."""
    w, g, _, dm, _ = _case()
    J = dv.jacobian_forward(g, w.m, w.src, w.rec, dm, stencil=stencil, w27=w27)
    e = 1e-4
    Fp = dv.forward_data(g, w.m + e * dm, w.src, w.rec, stencil=stencil, w27=w27)
    Fm = dv.forward_data(g, w.m - e * dm, w.src, w.rec, stencil=stencil, w27=w27)
    fd = (Fp - Fm) / (2 * e)
    assert np.linalg.norm(J - fd) <= 1e-6 * np.linalg.norm(J)


def test_jacobian_taylor_remainder_is_second_order():
    """Taylor test (Validation section) of the forward map: ||F(m + h dm) -
    F(m) - h J dm|| decays like h^2, ||F(m + h dm) - F(m)|| like h."""
    w, g, _, dm, _ = _case(seed=41)
    J = dv.jacobian_forward(g, w.m, w.src, w.rec, dm)
    F0 = dv.forward_data(g, w.m, w.src, w.rec)
    hs = np.array([1e-1, 5e-2, 2.5e-2, 1.25e-2]) * 0.2
    r0, r1 = [], []
    for h in hs:
        Fh = dv.forward_data(g, w.m + h * dm, w.src, w.rec)
        r0.append(np.linalg.norm(Fh - F0))
        r1.append(np.linalg.norm(Fh - F0 - h * J))
    assert abs(np.polyfit(np.log(hs), np.log(r0), 1)[0] - 1.0) < 0.1
    assert abs(np.polyfit(np.log(hs), np.log(r1), 1)[0] - 2.0) < 0.1


@pytest.mark.parametrize("stencil,w27", STENCILS)
def test_jacobian_adjoint_identity(stencil, w27):
    """<J x, y> = <x, J^* y> (real inner products; the paper's adjoint-test
    table: Jacobian row) with exact solves: to 1e-12."""
    w, g, _, x, rng = _case(seed=42)
    y = (rng.standard_normal((len(w.src), len(w.rec)))
         + 1j * rng.standard_normal((len(w.src), len(w.rec))))
    Jx = dv.jacobian_forward(g, w.m, w.src, w.rec, x, stencil=stencil, w27=w27)
    Jty = dv.jacobian_adjoint(g, w.m, w.src, w.rec, y, stencil=stencil, w27=w27)
    lhs = float(np.real(np.vdot(y, Jx)))
    rhs = float(np.sum(x * Jty))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Jx) * np.linalg.norm(y)


def test_jacobian_adjoint_of_residual_is_the_gradient():
    """grad f = J^* (P_r u - d) (Table derivstuff): equals the gradient of
    the misfit module, itself pinned by exact central differences."""
    w, g, d, _, _ = _case(seed=43)
    f, grad, us, _ = fwi.misfit_gradient(g, w.m, w.src, w.rec, d)
    r = np.stack([fwi.sample(u, w.rec) for u in us]) - d
    Jtr = dv.jacobian_adjoint(g, w.m, w.src, w.rec, r)
    assert np.linalg.norm(Jtr - grad) <= 1e-12 * np.linalg.norm(grad)


def test_gauss_newton_matches_dense_jacobian_from_finite_differences():
    """H_GN dm vs Re(J^H J) dm with J assembled column by column from central
    differences of the forward map (one re-solve pair per cell) on a tiny
    grid: brute force, no adjoint state involved."""
    w = workloads.layered_random_workload((7, 6, 6), 25.0, 1, 6.0, nsrc_xy=(1, 1),
                                          nrec_xy=(3, 2), seed=44)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    rng = np.random.default_rng(44)
    dm = rng.standard_normal(g.n) * w.m
    cols = []
    for k in range(g.N):
        e = np.zeros(g.N)
        e[k] = 1e-4 * w.m.ravel()[k]
        e = e.reshape(g.n)
        Fp = dv.forward_data(g, w.m + e, w.src, w.rec)
        Fm = dv.forward_data(g, w.m - e, w.src, w.rec)
        cols.append(((Fp - Fm) / (2 * e.ravel()[k])).ravel())
    Jd = np.stack(cols, axis=1)
    ref = np.real(Jd.conj().T @ (Jd @ dm.ravel())).reshape(g.n)
    H = dv.hessian_gn(g, w.m, w.src, w.rec, dm)
    assert np.linalg.norm(H - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("stencil,w27", STENCILS)
def test_gauss_newton_symmetric_and_equals_norm_of_jx(stencil, w27):
    w, g, _, x, rng = _case(seed=45)
    y = workloads.gaussian_random_field(rng, g.n, 2.0) * w.m
    Hx = dv.hessian_gn(g, w.m, w.src, w.rec, x, stencil=stencil, w27=w27)
    Hy = dv.hessian_gn(g, w.m, w.src, w.rec, y, stencil=stencil, w27=w27)
    a, b = float(np.sum(Hx * y)), float(np.sum(x * Hy))
    assert abs(a - b) <= 1e-12 * np.linalg.norm(Hx) * np.linalg.norm(y)
    Jx = dv.jacobian_forward(g, w.m, w.src, w.rec, x, stencil=stencil, w27=w27)
    jj = float(np.vdot(Jx, Jx).real)
    assert abs(float(np.sum(x * Hx)) - jj) <= 1e-12 * jj


@pytest.mark.parametrize("stencil,w27", STENCILS)
def test_full_hessian_matches_central_difference_of_gradient(stencil, w27):
    """grad^2 f dm vs (grad f(m + e dm) - grad f(m - e dm)) / 2e, gradients
    by exact solves (the gradient is pinned by exact central differences of
    f): O(e^2) agreement."""
    w, g, d, dm, _ = _case(seed=46)
    # data far from the model's so that the second-order term matters
    H = dv.hessian_full(g, w.m, w.src, w.rec, d, dm, stencil=stencil, w27=w27)
    e = 1e-4
    gp = fwi.misfit_gradient(g, w.m + e * dm, w.src, w.rec, d, stencil=stencil, w27=w27)[1]
    gm = fwi.misfit_gradient(g, w.m - e * dm, w.src, w.rec, d, stencil=stencil, w27=w27)[1]
    fd = (gp - gm) / (2 * e)
    assert np.linalg.norm(H - fd) <= 1e-6 * np.linalg.norm(fd)
    # the second-order term is not negligible here (the pin would miss it)
    Hgn = dv.hessian_gn(g, w.m, w.src, w.rec, dm, stencil=stencil, w27=w27)
    assert np.linalg.norm(H - Hgn) >= 1e-2 * np.linalg.norm(H)


@pytest.mark.parametrize("stencil,w27", STENCILS)
def test_full_hessian_symmetric(stencil, w27):
    """<H x, y> = <x, H y> (the paper's adjoint-test table: Hessian row)."""
    w, g, d, x, rng = _case(seed=47)
    y = workloads.gaussian_random_field(rng, g.n, 2.0) * w.m
    Hx = dv.hessian_full(g, w.m, w.src, w.rec, d, x, stencil=stencil, w27=w27)
    Hy = dv.hessian_full(g, w.m, w.src, w.rec, d, y, stencil=stencil, w27=w27)
    a, b = float(np.sum(Hx * y)), float(np.sum(x * Hy))
    assert abs(a - b) <= 1e-11 * np.linalg.norm(Hx) * np.linalg.norm(y)


@pytest.mark.parametrize("stencil,w27", STENCILS)
def test_full_hessian_at_zero_residual_is_gauss_newton(stencil, w27):
    """With d = F(m) the adjoint field vanishes and the full Hessian reduces
    to the Gauss-Newton Hessian."""
    w, g, _, dm, _ = _case(seed=48)
    d0 = dv.forward_data(g, w.m, w.src, w.rec, stencil=stencil, w27=w27)
    H = dv.hessian_full(g, w.m, w.src, w.rec, d0, dm, stencil=stencil, w27=w27)
    Hgn = dv.hessian_gn(g, w.m, w.src, w.rec, dm, stencil=stencil, w27=w27)
    assert np.linalg.norm(H - Hgn) <= 1e-12 * np.linalg.norm(Hgn)


def test_pairs_products_by_resolving():
    """Over (frequency, source) pairs with a mask, complex amplitudes and the
    1/|I| average: J dm per pair against a central difference of the pair's
    re-solved data, and the full Hessian against a central difference of
    the averaged gradient (pinned by re-solving in the misfit tests)."""
    w, g, _, dm, rng = _case(seed=49, nsrc=(3, 1))
    omegas = [2 * np.pi * 5.0, 2 * np.pi * 6.5]
    ns, nr = len(w.src), len(w.rec)
    d = (rng.standard_normal((2, ns, nr)) + 1j * rng.standard_normal((2, ns, nr))) * 1e-4
    amp = rng.standard_normal((2, ns)) + 1j * rng.standard_normal((2, ns))
    mask = np.array([[True, False, True], [False, True, True]])
    J = dv.jacobian_forward_pairs(g, w.m, omegas, w.src, w.rec, dm, amp=amp, mask=mask)
    e = 1e-4
    for fi, om in enumerate(omegas):
        gf = replace(g, omega=om)
        for s in range(ns):
            if not mask[fi, s]:
                assert np.all(J[fi, s] == 0)
                continue
            Fp = dv.forward_data(gf, w.m + e * dm, w.src[s:s + 1], w.rec, amp=amp[fi, s:s + 1])
            Fm = dv.forward_data(gf, w.m - e * dm, w.src[s:s + 1], w.rec, amp=amp[fi, s:s + 1])
            fd = ((Fp - Fm) / (2 * e))[0]
            assert np.linalg.norm(J[fi, s] - fd) <= 1e-6 * np.linalg.norm(fd)
    H = dv.hessian_full_pairs(g, w.m, omegas, w.src, w.rec, d, dm, amp=amp, mask=mask,
                              renormalise=True)
    gp = fwi.misfit_gradient_pairs(g, w.m + e * dm, omegas, w.src, w.rec, d, amp=amp, mask=mask,
                                   renormalise=True)[1]
    gm = fwi.misfit_gradient_pairs(g, w.m - e * dm, omegas, w.src, w.rec, d, amp=amp, mask=mask,
                                   renormalise=True)[1]
    fd = (gp - gm) / (2 * e)
    assert np.linalg.norm(H - fd) <= 1e-6 * np.linalg.norm(fd)
