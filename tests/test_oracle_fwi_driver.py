"""Pins of the inversion-driver oracle (frequency continuation, stochastic
source subsets, box-constrained L-BFGS): the source generator against its
published outputs, uniformity of the subsets, the band partition of the 2D
example, the L-BFGS on problems whose solution is known (an unconstrained
quadratic, a bound-constrained quadratic solved by enumerating the active
sets, a bounded Rosenbrock valley), its failure path, and the driver on a
tiny inversion (reduction to one plain L-BFGS run, clamped points, subset
growth, misfit reduction)."""
import itertools
from pathlib import Path

import numpy as np
import pytest

from oracle import fwi, fwi_driver as drv
from oracle import operators as ops
import workloads

GOLDEN = Path(__file__).parent / "golden"


def test_splitmix64_published_outputs():
    want = [int(s) for s in (GOLDEN / "splitmix64_seed1234567.txt").read_text().split("\n")
            if s and not s.startswith("#")]
    d = drv.Draws(1234567)
    assert [d.next() for _ in range(5)] == want


def test_subsets_are_uniform_and_valid():
    """Every 2-of-5 subset is equally likely (chi-square over 20,000 draws,
    9 degrees of freedom, 0.1 % critical value 27.9); subsets are sorted,
    distinct and in range; drawing every source consumes nothing."""
    d = drv.Draws(7)
    counts = {}
    for _ in range(20000):
        s = drv.draw_subset(d, 5, 2)
        assert s == sorted(set(s)) and all(0 <= i < 5 for i in s) and len(s) == 2
        counts[tuple(s)] = counts.get(tuple(s), 0) + 1
    assert len(counts) == 10
    chi2 = sum((c - 2000) ** 2 / 2000 for c in counts.values())
    assert chi2 < 27.9
    # each index's inclusion frequency is p / n
    d = drv.Draws(8)
    inc = np.zeros(9)
    for _ in range(9000):
        inc[drv.draw_subset(d, 9, 4)] += 1
    assert np.all(np.abs(inc / 9000 - 4 / 9) < 0.02)
    c = d.counter
    assert drv.draw_subset(d, 6, 6) == list(range(6)) and drv.draw_subset(d, 6, 9) == list(range(6))
    assert d.counter == c


def test_bands_of_the_2d_example():
    assert drv.bands(10, 4, 2) == [[0, 1, 2, 3], [2, 3, 4, 5], [4, 5, 6, 7], [6, 7, 8, 9]]
    assert drv.bands(11, 4, 2)[-1] == [8, 9, 10] and len(drv.bands(11, 4, 2)) == 5
    assert drv.bands(3, 4, 2) == [[0, 1, 2]]
    assert drv.bands(6, 2, 0) == [[0, 1], [2, 3], [4, 5]]
    assert drv.bands(5, 1, 0) == [[i] for i in range(5)]  # one frequency at a time (the 3D example)
    with pytest.raises(ValueError):
        drv.bands(5, 2, 2)


def _quadratic(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.geomspace(1.0, cond, n)) @ Q.T
    b = rng.standard_normal(n)
    return A, b, (lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b))


def test_lbfgs_unconstrained_quadratic():
    A, b, fg = _quadratic(8, 100.0, 1)
    xs = np.linalg.solve(A, b)
    log = []
    x, failed = drv.projected_lbfgs(fg, np.zeros(8), -1e3, 1e3, 80, 5, 0.5, gtol=1e-7, log=log)
    assert not failed and len(log) < 80  # stopped by the gradient tolerance
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)  # |x - x*| <= |g| / lambda_min
    fs = [r["f"] for r in log] + [log[-1]["f_new"]]
    assert all(b2 <= a2 for a2, b2 in zip(fs, fs[1:]))  # Armijo: monotone
    # without memory it is projected steepest descent: still converges on a well-conditioned problem
    A2, b2_, fg2 = _quadratic(6, 4.0, 2)
    x2, _ = drv.projected_lbfgs(fg2, np.zeros(6), -1e3, 1e3, 300, 0, 0.5, max_ls=50, gtol=1e-9)
    assert np.linalg.norm(x2 - np.linalg.solve(A2, b2_)) <= 1e-5


def _box_qp_bruteforce(A, b, lo, hi):
    """Minimiser of 1/2 x'Ax - b'x on [lo, hi]^n: the unique active-set
    assignment (free / at lo / at hi) whose solution satisfies the KKT
    conditions."""
    n = len(b)
    best = None
    for act in itertools.product((0, 1, 2), repeat=n):
        x = np.array([lo if a == 1 else hi if a == 2 else 0.0 for a in act])
        F = [i for i in range(n) if act[i] == 0]
        if F:
            B = [i for i in range(n) if act[i] != 0]
            x[F] = np.linalg.solve(A[np.ix_(F, F)], b[F] - A[np.ix_(F, B)] @ x[B])
        gr = A @ x - b
        ok = all(lo - 1e-12 <= x[i] <= hi + 1e-12 for i in F)
        ok &= all(gr[i] >= -1e-12 for i in range(n) if act[i] == 1)
        ok &= all(gr[i] <= 1e-12 for i in range(n) if act[i] == 2)
        if ok:
            best = x
    return best


def test_lbfgs_bound_constrained_quadratic():
    A, b, fg = _quadratic(5, 20.0, 3)
    b = 3.0 * b
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    lo, hi = -0.4, 0.5
    xs = _box_qp_bruteforce(A, b, lo, hi)
    assert np.sum((xs <= lo) | (xs >= hi)) >= 2  # the bounds bind
    x, _ = drv.projected_lbfgs(fg, np.zeros(5), lo, hi, 200, 5, 0.2, gtol=1e-12)
    assert np.abs(x - xs).max() <= 1e-7
    # per-point bounds (an array), one variable clamped (lo = hi)
    lo_a = np.full(5, lo)
    hi_a = np.full(5, hi)
    lo_a[2] = hi_a[2] = 0.1
    x, _ = drv.projected_lbfgs(fg, np.zeros(5), lo_a, hi_a, 200, 5, 0.2)
    assert x[2] == 0.1 and np.all(x >= lo_a) and np.all(x <= hi_a)


def test_lbfgs_bounded_rosenbrock():
    """Rosenbrock's valley with x <= 0.5: the minimiser is (0.5, 0.25), where
    the x-gradient -1 points out of the box."""
    def fg(z):
        x, y = z
        return ((1 - x) ** 2 + 100 * (y - x * x) ** 2,
                np.array([-2 * (1 - x) - 400 * x * (y - x * x), 200 * (y - x * x)]))
    z, failed = drv.projected_lbfgs(fg, np.array([-1.2, 1.0]), np.array([-2.0, -2.0]), np.array([0.5, 2.0]),
                                    300, 5, 0.5, gtol=1e-12)
    assert np.abs(z - [0.5, 0.25]).max() <= 1e-6
    z, _ = drv.projected_lbfgs(fg, np.array([-1.2, 1.0]), -2.0, 2.0, 400, 5, 0.5, gtol=1e-12)
    assert np.abs(z - [1.0, 1.0]).max() <= 1e-5


def test_lbfgs_failed_line_search_keeps_the_iterate():
    """A gradient of the wrong sign: no trial satisfies Armijo, the iterate stays."""
    fg = lambda x: (0.5 * x @ x, -x)
    x0 = np.array([1.0, -2.0])
    log = []
    x, failed = drv.projected_lbfgs(fg, x0, -5.0, 5.0, 10, 3, 1.0, max_ls=4, log=log)
    assert failed and np.array_equal(x, x0) and len(log) == 1 and log[0]["trials"] == 4
    assert not log[0]["accepted"]


def _tiny(seed=90):
    n, npml = (14, 13, 12), 3
    w = workloads.layered_random_workload(n, 25.0, npml, 6.0, nsrc_xy=(2, 2), nrec_xy=(4, 4), seed=seed)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    m_true = w.m.copy()
    rng = np.random.default_rng(seed)
    I, J, K = np.indices(n)
    blob = np.exp(-((I - 7) ** 2 + (J - 6) ** 2 + (K - 7) ** 2) / 8.0)
    m_true = m_true * (1.0 + 0.15 * blob)
    m0 = w.m.copy()
    omegas = 2 * np.pi * np.array([4.0, 5.0, 6.0])
    amp = np.ones((3, len(w.src)), np.complex128)
    d = np.zeros((3, len(w.src), len(w.rec)), np.complex128)
    for fi, om in enumerate(omegas):
        from dataclasses import replace
        solve = fwi.LUSolver(replace(g, omega=om), m_true)
        for s, p in enumerate(w.src):
            d[fi, s] = fwi.sample(solve(fwi.point_source(g, p)), w.rec)
    lo, hi = 0.8 * m0.min(), 1.2 * m_true.max()
    return w, g, m_true, m0, omegas, amp, d, lo, hi, rng


def test_driver_single_band_is_one_lbfgs_run():
    """One band over every frequency, every source, one draw: the driver is
    projected_lbfgs on the averaged objective over all pairs."""
    w, g, m_true, m0, omegas, amp, d, lo, hi, _ = _tiny()
    kw = dict(amp=amp, mask=None, renormalise=True)
    fg = lambda x: fwi.misfit_gradient_pairs(g, x, omegas, w.src, w.rec, d, **kw)[:2]
    x_ref, _ = drv.projected_lbfgs(fg, m0, lo, hi, 3, 5, drv.default_step0(lo, hi))
    x = drv.fwi_invert(g, m0, lo, hi, omegas, w.src, w.rec, d, amp=amp, band_size=3, band_overlap=0, r_sub=3)
    assert np.array_equal(x, x_ref)


def test_driver_reduces_misfit_and_respects_bounds():
    w, g, m_true, m0, omegas, amp, d, lo, hi, _ = _tiny()
    lo_a = np.full(g.n, lo)
    hi_a = np.full(g.n, hi)
    lo_a[:, :, :4] = hi_a[:, :, :4] = m0[:, :, :4]  # a clamped layer (the water of the 3D example)
    log = []
    x = drv.fwi_invert(g, m0, lo_a, hi_a, omegas, w.src, w.rec, d, amp=amp, band_size=2, band_overlap=1,
                       r_sub=4, log=log)
    assert [e["band"] for e in log] == [0, 1]
    assert np.array_equal(x[:, :, :4], m0[:, :, :4]) and np.all(x >= lo_a) and np.all(x <= hi_a)
    f0 = fwi.misfit_gradient_pairs(g, m0, omegas, w.src, w.rec, d, amp=amp, renormalise=True)[0]
    f1 = fwi.misfit_gradient_pairs(g, x, omegas, w.src, w.rec, d, amp=amp, renormalise=True)[0]
    assert f1 < 0.5 * f0
    for e in log:
        fs = [s["f"] for s in e["steps"]]
        assert all(b <= a for a, b in zip(fs, fs[1:]))


def test_driver_stochastic_subsets_and_growth():
    """Subsets of p = 1 of 4 sources, r_sub ceil(N_s / p) iterations each; a
    line search that cannot succeed (max_ls = 1 with an oversized first step)
    grows p by batch_increase for the next draw."""
    w, g, m_true, m0, omegas, amp, d, lo, hi, _ = _tiny()
    log = []
    drv.fwi_invert(g, m0, lo, hi, omegas, w.src, w.rec, d, amp=amp, band_size=3, band_overlap=0, r_sub=1,
                   batch=1, subproblems=3, batch_increase=2, seed=5, max_ls=1, step0=50.0 * (hi - lo), log=log)
    dr = drv.Draws(5)
    p = 1
    for e in log:
        assert e["sources"] == drv.draw_subset(dr, 4, p)
        assert e["iters"] == drv.iterations(1, 4, p)
        p = min(4, p + 2) if e["failed"] else p
    assert log[0]["failed"] and len(log[1]["sources"]) == 3
