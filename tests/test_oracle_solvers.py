"""Pins of the oracle's GMRES / FGMRES / ML-GMRES against brute force,
library routines, invariants and the paper's printed iteration counts."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import krylov, mlgmres, fwi
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cplx(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_gmres_full_dimension_equals_direct_solve():
    """GMRES(k = n) on a tiny dense nonsymmetric complex system is exact."""
    rng = np.random.default_rng(10)
    for n in (3, 8, 17):
        A = _cplx(rng, (n, n)) + 4 * np.eye(n)
        b = _cplx(rng, n)
        x, info = krylov.gmres(lambda v: A @ v, b, k=n, cycles=1)
        assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)


def test_gmres_on_assembled_helmholtz_matches_lu():
    """Restarted GMRES on a 4^3 Helmholtz system with a layer vs a dense
    direct solve of the assembled matrix."""
    g = ops.make_grid((4, 4, 4), 10.0, 1, 2 * np.pi * 5, 2000.0)
    m = np.full(g.n, 1 / 2000.0 ** 2)
    H = ops.assemble7(g, m).toarray()
    rng = np.random.default_rng(11)
    b = _cplx(rng, g.n)
    x, info = krylov.gmres(lambda v: ops.apply7(g, m, v), b, k=10, cycles=200,
                           tol=1e-13)
    xd = np.linalg.solve(H, b.ravel()).reshape(g.n)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_arnoldi_relation_and_orthonormality():
    rng = np.random.default_rng(12)
    n, k = 40, 12
    A = _cplx(rng, (n, n))
    V, Hb = krylov.arnoldi_relation(lambda v: A @ v, _cplx(rng, n), k)
    assert np.abs(A @ V[:, :k] - V @ Hb).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(V.conj().T @ V - np.eye(k + 1)).max() <= 1e-12


def test_fgmres_with_fixed_linear_preconditioner_equals_right_gmres():
    """With a fixed linear M, FGMRES and right-preconditioned GMRES build the
    same Krylov space: identical iterates after each cycle."""
    rng = np.random.default_rng(13)
    n = 30
    A = _cplx(rng, (n, n)) + 6 * np.eye(n)
    Mm = np.eye(n) + 0.1 * _cplx(rng, (n, n))
    b = _cplx(rng, n)
    for cyc in (1, 2, 3):
        x1, _ = krylov.fgmres(lambda v: A @ v, b, M=lambda v: Mm @ v, k=5,
                              cycles=cyc)
        x2, _ = krylov.gmres(lambda v: A @ v, b, M=lambda v: Mm @ v, k=5,
                             cycles=cyc)
        assert np.linalg.norm(x1 - x2) <= 1e-11 * np.linalg.norm(x2)


def test_gmres20_small_config_vs_scipy_and_splu():
    """A reduced version of the 32^3 complex128 GMRES(20) case (16^3, same
    physics): the oracle's restarted GMRES(20) converges to 1e-6 and its
    iterate after a fixed number of cycles matches SciPy's GMRES(20) (same
    Krylov spaces); the converged solution matches SuperLU."""
    w = workloads.c1_small()
    n = (16, 16, 16)
    v = w.v[8:24, 8:24, 8:24]
    g = ops.make_grid(n, w.h, 4, w.omega, float(v.max()))
    m = 1.0 / v ** 2
    q = fwi.point_source(g, (8, 8, 8))
    A = lambda x: ops.apply7(g, m, x)
    x3, _ = krylov.gmres(A, q, k=20, cycles=3)
    H = ops.assemble7(g, m)
    xs, _ = spla.gmres(H, q.ravel(), restart=20, maxiter=3, rtol=1e-30, atol=0)
    assert np.linalg.norm(x3.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)
    x, info = krylov.gmres(A, q, k=20, cycles=500, tol=1e-10)
    assert info["relres"] <= 1e-10
    xe = fwi.LUSolver(g, m)(q)
    assert np.linalg.norm(x - xe) <= 1e-7 * np.linalg.norm(xe)


# ----------------------------------------------------------------------------
# multigrid pieces
# ----------------------------------------------------------------------------

def test_prolongation_reproduces_linear_functions():
    for nf in [(9, 10, 7), (8, 8, 8)]:
        nc = tuple(a // 2 + 1 for a in nf)
        Ic = np.meshgrid(*[2.0 * np.arange(a) for a in nc], indexing="ij")
        If = np.meshgrid(*[np.arange(a, dtype=float) for a in nf], indexing="ij")
        lin_c = 1.5 + 0.3 * Ic[0] - 0.7 * Ic[1] + 0.2 * Ic[2]
        lin_f = 1.5 + 0.3 * If[0] - 0.7 * If[1] + 0.2 * If[2]
        assert np.abs(mlgmres.prolong(lin_c, nf) - lin_f).max() <= 1e-13


def test_restriction_is_full_weighting_over_eight():
    """R = P^T / 8 equals the textbook full-weighting stencil
    (1/8) sum_{d in {-1,0,1}^3} prod_a (1 - |d_a|/2) r(2I + d), written out
    point by point (fine nodes outside the grid contribute zero)."""
    rng = np.random.default_rng(14)
    nf = (9, 8, 7)
    r = _cplx(rng, nf)
    Rr = mlgmres.restrict(r)
    nc = tuple(a // 2 + 1 for a in nf)
    assert Rr.shape == nc
    ref = np.zeros(nc, complex)
    for I in np.ndindex(*nc):
        acc = 0.0
        for d in np.ndindex(3, 3, 3):
            dd = np.array(d) - 1
            p = 2 * np.array(I) + dd
            if np.all(p >= 0) and np.all(p < np.array(nf)):
                acc += np.prod(1 - np.abs(dd) / 2.0) * r[tuple(p)]
        ref[I] = acc / 8.0
    assert np.abs(Rr - ref).max() <= 1e-14 * np.abs(ref).max()


def test_inject_model_and_coarse_grid():
    mf = np.arange(9 * 8 * 5, dtype=float).reshape(9, 8, 5)
    mc = mlgmres.inject_model(mf)
    assert mc.shape == (5, 5, 3)
    assert mc[2, 4, 1] == mf[4, 7, 2]  # 2*4 = 8 clipped to 7
    g = ops.make_grid((9, 8, 5), 10.0, 2, 3.0, 2000.0)
    gc = ops.coarsen(g)
    assert gc.n == (5, 5, 3) and gc.h == 20.0 and gc.stride == 2
    # coarse profile = fine profile at fine coordinates 2I, 2I +- 1
    assert np.allclose(ops.stretch(gc, 0, np.arange(5) + 0.5),
                       ops.stretch(g, 0, 2 * np.arange(5) + 1.0))


def test_memory_bound_is_26_vectors():
    """The paper's peak-memory formula at (3,5,3,5), k = 5 gives 26 N."""
    assert mlgmres.workspace_vectors(mlgmres.MLOptions()) == 26.0


def _constant_case(nl, ppw, v0=2000.0, f=5.0):
    n = nl * ppw + 1 + 2 * ppw
    h = v0 / (f * ppw)
    g = ops.make_grid((n, n, n), h, ppw, 2 * np.pi * f, v0)
    m = np.full(g.n, 1 / v0 ** 2)
    q = fwi.point_source(g, (n // 2,) * 3)
    return g, m, q


def test_mlgmres_converges_and_certifies():
    """ML-GMRES on a constant-velocity 8-ppw problem reaches rel. res. 1e-6
    in a few outer cycles; its solution matches a tight GMRES solve."""
    g, m, q = _constant_case(2, 8)
    x, info = mlgmres.mlgmres_solve(g, m, q, tol=1e-6)
    r = np.linalg.norm(q - ops.apply7(g, m, x)) / np.linalg.norm(q)
    assert r <= 1e-6 and info["cycles"] <= 3
    xe, _ = krylov.gmres(lambda v: ops.apply7(g, m, v), q, k=30, cycles=3000,
                         tol=1e-11)
    assert np.linalg.norm(x - xe) <= 1e-4 * np.linalg.norm(xe)
    # adjoint solve with the adjoint operators on every level
    y, info = mlgmres.mlgmres_solve(g, m, q, tol=1e-6, adjoint=True)
    r = np.linalg.norm(q - ops.apply7(g, m, y, True)) / np.linalg.norm(q)
    assert r <= 1e-6


@pytest.mark.slow
def test_mlgmres_outer_cycles_vs_paper_table():
    """Paper, preconditioner-performance table: constant velocity, layer of
    one wavelength, FGMRES(5) to 1e-6 with (3,5,3,5).  Row n_lambda = 5:
    ppw 6 -> 2 cycles (43^3), ppw 8 -> 2 cycles (57^3).  Our 7-point
    discretisation differs from the paper's 27-point one, so we accept the
    printed count +- 1."""
    with open(os.path.join(GOLDEN, "precond_table.json")) as fh:
        table = json.load(fh)
    for row in table["rows"]:
        if row["n_lambda"] != 5 or row["ppw"] not in (6, 8):
            continue
        g, m, q = _constant_case(row["n_lambda"], row["ppw"])
        assert g.n[0] == row["grid"]
        x, info = mlgmres.mlgmres_solve(g, m, q, tol=1e-6)
        assert abs(info["cycles"] - row["outer_cycles"]) <= 1
        assert info["relres"] <= 1e-6
