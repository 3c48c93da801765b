"""Pins of the oracle's misfit and adjoint-state gradient: a zero-residual
special case, brute-force finite differences by re-solving, the exact
rank-one central difference, and the paper's Taylor test."""
import numpy as np

from oracle import operators as ops
from oracle import fwi
import workloads

W27 = (0.55, 0.3, 0.15, 0.62 - 0.0, 0.06, 0.0025, -0.001)


def _w27_valid(w):
    w = list(w)
    w[3] = 1.0 - 6 * w[4] - 12 * w[5] - 8 * w[6]
    w[0] = 1.0 - w[1] - w[2]
    return tuple(w)


def _small_fwi(seed=20, n=(14, 13, 12), npml=3, nsrc=(2, 2), nrec=(4, 4)):
    w = workloads.layered_random_workload(n, 25.0, npml, 6.0, nsrc_xy=nsrc,
                                          nrec_xy=nrec, seed=seed)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((len(w.src), len(w.rec))) * 1e-4 + \
        1j * rng.standard_normal((len(w.src), len(w.rec))) * 1e-4
    return w, g, d


def _interior_cells(g, rng, count):
    lo, hi = g.npml + 1, np.array(g.n) - g.npml - 1
    return [tuple(rng.integers(lo, hi[a]) for a in range(3)) for _ in range(count)]


def test_zero_residual_gives_zero_misfit_and_gradient():
    w, g, _ = _small_fwi()
    solve = fwi.LUSolver(g, w.m)
    us = [solve(fwi.point_source(g, p), False) for p in w.src]
    d = np.stack([fwi.sample(u, w.rec) for u in us])
    f, grad, _, _ = fwi.misfit_gradient(g, w.m, w.src, w.rec, d, solve=solve)
    assert f == 0.0
    assert np.abs(grad).max() == 0.0


def _brute_fd(g, m, k, eps, src, rec, d, stencil="7pt", w27=None):
    mp, mm = m.copy(), m.copy()
    mp[k] += eps
    mm[k] -= eps
    fp = fwi.objective(g, mp, src, rec, d, stencil=stencil, w27=w27)
    fm = fwi.objective(g, mm, src, rec, d, stencil=stencil, w27=w27)
    return (fp - fm) / (2 * eps)


def test_exact_central_difference_matches_resolving():
    """The Sherman-Morrison central difference equals the one obtained by
    re-solving at m +- eps e_k (7-point and 27-point)."""
    w, g, d = _small_fwi()
    rng = np.random.default_rng(21)
    for stencil, w27 in (("7pt", None), ("27pt", _w27_valid(W27))):
        solve = fwi.LUSolver(g, w.m, stencil, w27)
        f, grad, us, vs = fwi.misfit_gradient(g, w.m, w.src, w.rec, d,
                                              stencil=stencil, w27=w27,
                                              solve=solve)
        _, rs = fwi.misfit(us, d, w.rec)
        for k in _interior_cells(g, rng, 2):
            eps = 1e-2 * w.m[k]
            ex = fwi.exact_central_difference(g, w.m, k, eps, us, rs, w.rec,
                                              solve, stencil, w27)
            bf = _brute_fd(g, w.m, k, eps, w.src, w.rec, d, stencil, w27)
            assert abs(ex - bf) <= 1e-6 * abs(ex) + 1e-12 * f / w.m[k]


def test_gradient_matches_exact_central_difference():
    """Adjoint-state gradient vs the exact central FD (eps = 1e-3 m_k) on
    random interior cells: agreement to the O(eps^2) truncation (1e-6)."""
    w, g, d = _small_fwi(seed=22)
    rng = np.random.default_rng(23)
    for stencil, w27 in (("7pt", None), ("27pt", _w27_valid(W27))):
        solve = fwi.LUSolver(g, w.m, stencil, w27)
        f, grad, us, vs = fwi.misfit_gradient(g, w.m, w.src, w.rec, d,
                                              stencil=stencil, w27=w27,
                                              solve=solve)
        _, rs = fwi.misfit(us, d, w.rec)
        gmax = np.abs(grad).max()
        for k in _interior_cells(g, rng, 8):
            eps = 1e-3 * w.m[k]
            fd = fwi.exact_central_difference(g, w.m, k, eps, us, rs, w.rec,
                                              solve, stencil, w27)
            assert abs(fd - grad[k]) <= 1e-6 * max(abs(fd), 1e-3 * gmax)


def test_taylor_remainders_first_and_second_order():
    """Paper's Taylor test (Validation section): along a random dm the
    zeroth-order remainder decays like h and the first-order one like h^2."""
    w, g, d = _small_fwi(seed=24, n=(12, 12, 12))
    rng = np.random.default_rng(25)
    dm = rng.standard_normal(g.n) * w.m * 0.05
    hs = np.array([1e-1, 5e-2, 2.5e-2, 1.25e-2])
    r0, r1 = fwi.taylor_remainders(g, w.m, dm, w.src, w.rec, d, hs)
    s0 = np.polyfit(np.log(hs), np.log(r0), 1)[0]
    s1 = np.polyfit(np.log(hs), np.log(r1), 1)[0]
    assert abs(s0 - 1.0) < 0.1
    assert abs(s1 - 2.0) < 0.1


def test_sampling_adjoint_identity():
    rng = np.random.default_rng(26)
    n = (6, 7, 8)
    rec = np.array([[1, 2, 3], [4, 4, 4], [1, 2, 3]])
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    a = np.vdot(r, fwi.sample(u, rec))
    b = np.vdot(fwi.sample_adjoint(n, rec, r), u)
    assert abs(a - b) <= 1e-14 * abs(a)


def test_pairs_objective_gradient_by_resolving():
    """Sum over (frequency, source) pairs with a mask, complex amplitudes and
    the 1/|I| average of the selected pairs: the gradient equals a central
    difference of the objective re-solved from scratch pair by pair
    (7-point and 27-point)."""
    from dataclasses import replace
    w, g, _ = _small_fwi(seed=24, nsrc=(3, 1))
    rng = np.random.default_rng(24)
    omegas = [2 * np.pi * 5.0, 2 * np.pi * 6.5]
    ns, nr = len(w.src), len(w.rec)
    d = (rng.standard_normal((2, ns, nr)) + 1j * rng.standard_normal((2, ns, nr))) * 1e-4
    amp = rng.standard_normal((2, ns)) + 1j * rng.standard_normal((2, ns))
    mask = np.array([[True, False, True], [True, True, False]])

    def objective(m, stencil, w27):
        tot = 0.0
        for fi, om in enumerate(omegas):
            gf = replace(g, omega=om)
            solve = fwi.LUSolver(gf, m, stencil, w27)
            for s in range(ns):
                if mask[fi, s]:
                    u = solve(fwi.point_source(gf, w.src[s], amp[fi, s]))
                    r = fwi.sample(u, w.rec) - d[fi, s]
                    tot += 0.5 * float(np.vdot(r, r).real)
        return tot / mask.sum()

    for stencil, w27 in (("7pt", None), ("27pt", _w27_valid(W27))):
        f, grad, us, vs = fwi.misfit_gradient_pairs(g, w.m, omegas, w.src, w.rec, d, amp=amp,
                                                    mask=mask, renormalise=True, stencil=stencil,
                                                    w27=w27)
        assert sorted(us) == [(0, 0), (0, 2), (1, 0), (1, 1)]
        assert abs(f - objective(w.m, stencil, w27)) <= 1e-12 * f
        for k in _interior_cells(g, rng, 3):
            eps = 1e-4 * w.m[k]
            mp, mm = w.m.copy(), w.m.copy()
            mp[k] += eps
            mm[k] -= eps
            fd = (objective(mp, stencil, w27) - objective(mm, stencil, w27)) / (2 * eps)
            assert abs(grad[k] - fd) <= 1e-6 * np.abs(grad).max()
