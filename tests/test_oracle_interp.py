"""Pins of the off-grid interpolation oracle (Kaiser-windowed sinc sources
and receivers): the on-node special case equals the point source / sampling
of the misfit module, the window's closed form, the adjoint identity, the
interpolation of band-limited plane waves within the spectral error bound,
the fitted window shape, and the gradient with off-grid geometry against a
central difference of the objective re-solved from scratch."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import fwi, interp
from oracle import operators as ops
import workloads

R, B = workloads.SINC_RADIUS, workloads.SINC_KAISER_B


def test_on_node_positions_reduce_to_point_source_and_sampling():
    g = ops.make_grid((12, 11, 10), 20.0, 2, 2 * np.pi * 5, 3000.0)
    rng = np.random.default_rng(1)
    u = workloads.random_complex(rng, g.n)
    pts = np.array([[5, 4, 3], [0, 0, 0], [11, 10, 9], [6, 2, 8]])
    for p in pts:
        assert np.array_equal(interp.source(g, p.astype(float), R, B, 2 - 1j),
                              fwi.point_source(g, p, 2 - 1j))
    assert np.array_equal(interp.sample(u, pts.astype(float), R, B), fwi.sample(u, pts))
    r = workloads.random_complex(rng, len(pts))
    assert np.allclose(interp.sample_adjoint(g.n, pts.astype(float), R, B, r),
                       fwi.sample_adjoint(g.n, pts, r), rtol=0, atol=0)


def test_kaiser_window_closed_form():
    t = np.array([-R, -1.5, 0.0, 0.7, R, R + 0.1])
    w = interp.kaiser(t, R, B)
    assert w[2] == 1.0 and w[-1] == 0.0
    assert np.isclose(w[0], 1.0 / np.i0(B)) and np.isclose(w[4], 1.0 / np.i0(B))
    assert np.isclose(w[1], np.i0(B * np.sqrt(1 - (1.5 / R) ** 2)) / np.i0(B))
    # sinc factor: weights of an on-node position vanish away from it
    nodes, ws = interp.weights_1d(7.0, 20, R, B)
    assert np.allclose(ws[nodes != 7], 0.0) and ws[nodes == 7][0] == 1.0
    # nodes outside the grid are dropped
    nodes, ws = interp.weights_1d(1.3, 20, R, B)
    assert nodes.min() == 0 and len(nodes) == 2 + R


def test_adjoint_identity():
    rng = np.random.default_rng(2)
    n = (14, 13, 12)
    pos = rng.uniform([0.5, 0.5, 0.5], [12.5, 11.5, 10.5], size=(7, 3))
    u = workloads.random_complex(rng, n)
    r = workloads.random_complex(rng, 7)
    a = np.vdot(r, interp.sample(u, pos, R, B))
    b = np.vdot(interp.sample_adjoint(n, pos, R, B, r), u)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_plane_wave_interpolation_within_spectral_bound():
    """A plane wave sampled at 8 points per wavelength is interpolated at
    off-grid points (away from the grid edge) to within three times the
    window's 1D spectral error up to that wavenumber (tensor product)."""
    rng = np.random.default_rng(3)
    n = (24, 24, 24)
    kvec = 2 * np.pi / 8 * np.array([0.6, 0.64, 0.48])
    idx = np.indices(n).reshape(3, -1).T
    u = np.exp(1j * idx @ kvec).reshape(n)
    pos = rng.uniform(R + 1, 24 - R - 2, size=(40, 3))
    got = interp.sample(u, pos, R, B)
    ref = np.exp(1j * pos @ kvec)
    bound = 3 * interp.spectral_error(R, B, np.abs(kvec).max())
    assert np.abs(got - ref).max() <= bound
    assert bound < 1.5e-2  # the fitted window is within 0.5 % per axis at this sampling


def test_fitted_window_shape():
    """The stored b is the search's optimum: spectral error below 0.9 % at
    three points per wavelength, larger at nearby shapes."""
    kmax = 2 * np.pi / 3
    e = interp.spectral_error(R, B, kmax)
    assert e < 9e-3
    assert interp.spectral_error(R, B - 0.3, kmax) > e and interp.spectral_error(R, B + 0.3, kmax) > e
    assert abs(interp.fit_kaiser_b(R, kmax) - B) < 1e-6


def test_offgrid_gradient_by_resolving():
    """Misfit gradient with off-grid sources and receivers, two frequencies,
    masked pairs and 1/#pairs, against a central difference of the
    objective re-solved from scratch (7-point and 27-point)."""
    w = workloads.layered_random_workload((16, 15, 14), 25.0, 3, 6.0, nsrc_xy=(2, 1), seed=60)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    rng = np.random.default_rng(60)
    src = np.array([[6.3, 7.7, 4.2], [9.6, 6.1, 4.5]])
    rec = rng.uniform([4.0, 4.0, 3.5], [11.0, 10.0, 4.5], size=(9, 3))
    omegas = [2 * np.pi * 5.0, 2 * np.pi * 6.5]
    d = (rng.standard_normal((2, 2, 9)) + 1j * rng.standard_normal((2, 2, 9))) * 1e-4
    amp = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    mask = np.array([[True, True], [False, True]])
    w27 = workloads.W27_DEFAULT

    def objective(m, stencil, ww):
        tot = 0.0
        for fi, om in enumerate(omegas):
            gf = replace(g, omega=om)
            solve = fwi.LUSolver(gf, m, stencil, ww)
            for s in range(2):
                if mask[fi, s]:
                    u = solve(interp.source(gf, src[s], R, B, amp[fi, s]))
                    r = interp.sample(u, rec, R, B) - d[fi, s]
                    tot += 0.5 * float(np.vdot(r, r).real)
        return tot / mask.sum()

    for stencil, ww in (("7pt", None), ("27pt", w27)):
        f, grad = interp.misfit_gradient_pairs(g, w.m, omegas, src, rec, d, R, B, amp=amp, mask=mask,
                                               renormalise=True, stencil=stencil, w27=ww)
        assert abs(f - objective(w.m, stencil, ww)) <= 1e-12 * f
        lo, hi = g.npml + 1, np.array(g.n) - g.npml - 1
        for _ in range(3):
            k = tuple(rng.integers(lo, hi[a]) for a in range(3))
            eps = 1e-4 * w.m[k]
            mp, mm = w.m.copy(), w.m.copy()
            mp[k] += eps
            mm[k] -= eps
            fd = (objective(mp, stencil, ww) - objective(mm, stencil, ww)) / (2 * eps)
            assert abs(grad[k] - fd) <= 1e-6 * np.abs(grad).max()
