"""GPU parity of the two-dimensional operator (a grid with one node along its
first axis: the operator of the (n[1], n[2]) plane, as the 2.5D modelling
uses it) against the oracle's 2D assembly: helm_apply forward and adjoint in
both precisions on ragged shapes, and ML-GMRES solves against sparse LU."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import paper_1703_09268_amd as hx
from oracle import model25d as m25
from oracle import operators as ops

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(n, npml, seed, f=6.0, h=15.0):
    rng = np.random.default_rng(seed)
    v = 1500.0 + 2500.0 * rng.random((1,) + tuple(n))
    return rng, 1.0 / v ** 2, float(v.max()), 2 * np.pi * f, h


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("n,npml,nrhs", [((70, 45), 8, 3), ((37, 129), 5, 2), ((9, 600), 2, 1)])
def test_2d_apply_matches_oracle(dtype, adjoint, n, npml, nrhs):
    print(f"case 2d apply {dtype} adj={adjoint} n={n}", flush=True)
    rng, m, vref, omega, h = _case(n, npml, seed=sum(n))
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    rdt = torch.float32 if dtype == "c64" else torch.float64
    grid = hx.Grid(n=(1,) + n, h=h, npml=npml, v_ref=vref, dtype=dtype)
    m_t = torch.tensor(m, dtype=rdt, device=DEV)
    x = rng.standard_normal((nrhs, 1) + n) + 1j * rng.standard_normal((nrhs, 1) + n)
    x_t = torch.tensor(x, dtype=cdt, device=DEV)
    y = hx.helm_apply(grid, m_t, omega, x_t, adjoint=adjoint).cpu().numpy().astype(np.complex128)
    g = ops.make_grid((1,) + n, h, npml, omega, vref)
    H = m25.assemble2d(g, m_t.cpu().numpy().astype(np.float64), 0.0)
    if adjoint:
        H = H.conj().T
    xs = x_t.cpu().numpy().astype(np.complex128)
    tol = 1e-5 if dtype == "c64" else 1e-12
    for r in range(nrhs):
        ref = H @ xs[r].ravel()
        assert np.linalg.norm(y[r].ravel() - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("adjoint", [False, True])
def test_2d_solve_matches_lu(adjoint):
    """ML-GMRES (3 grids, the first axis kept at one node) to 1e-6 on a
    400 x 200 layered plane, four sources: certified by the oracle's FP64
    residual and within 1e-5 of the LU solution at tolerance 1e-9."""
    print(f"case 2d solve adj={adjoint}", flush=True)
    n, npml, h, f = (400, 200), 20, 10.0, 8.0
    rng = np.random.default_rng(3)
    depth = np.linspace(0.0, 1.0, n[1])
    v = (1500.0 + 2500.0 * depth)[None, None, :] * (1.0 + 0.05 * rng.standard_normal((1,) + n))
    omega = 2 * np.pi * f
    grid = hx.Grid(n=(1,) + n, h=h, npml=npml, v_ref=float(v.max()), dtype="c64")
    m_t = torch.tensor(1.0 / v ** 2, dtype=torch.float32, device=DEV)
    g = ops.make_grid((1,) + n, h, npml, omega, float(v.max()))
    q = np.zeros((4, 1) + n, np.complex128)
    for s, (j, k) in enumerate(((100, 25), (200, 25), (300, 25), (200, 100))):
        q[s] = m25.source2d(g, (j, k))
    q_t = torch.tensor(q, dtype=torch.complex64, device=DEV)
    u_t, info = hx.helm_solve(grid, m_t, omega, q_t, adjoint=adjoint, opts=hx.SolverOpts(tol=1e-6))
    H = m25.assemble2d(g, m_t.cpu().numpy().astype(np.float64), 0.0).tocsc()
    Hs = H.conj().T.tocsc() if adjoint else H
    u = u_t.cpu().numpy().astype(np.complex128)
    print("  cycles", [i.cycles for i in info], flush=True)
    # the FP64 iterate is certified at 1e-6; the returned complex64 field
    # adds at most ||H|| ||u|| 2^-23 / ||q|| from its rounding (||H||_2 bounded
    # by sqrt(||H||_1 ||H||_inf))
    Ha = abs(Hs)
    hnorm = float(np.sqrt(Ha.sum(axis=0).max() * Ha.sum(axis=1).max()))
    for s in range(4):
        rr = np.linalg.norm(q[s].ravel() - Hs @ u[s].ravel()) / np.linalg.norm(q[s])
        bound = 1e-6 + hnorm * np.linalg.norm(u[s]) * 2.0 ** -23 / np.linalg.norm(q[s])
        assert info[s].status == 0 and info[s].relres_fp64 <= 1e-6 and rr <= bound
    u_t, _ = hx.helm_solve(grid, m_t, omega, q_t, adjoint=adjoint, opts=hx.SolverOpts(tol=1e-9, max_cycles=200))
    lu = spla.splu(H)
    u = u_t.cpu().numpy().astype(np.complex128)
    for s in range(4):
        ue = lu.solve(q[s].ravel(), trans="H" if adjoint else "N")
        assert np.linalg.norm(u[s].ravel() - ue) <= 1e-5 * np.linalg.norm(ue)


def test_2d_grid_rules():
    m_t = torch.ones((1, 20, 20), dtype=torch.float32, device=DEV) * 1e-7
    x_t = torch.zeros((1, 20, 20), dtype=torch.complex64, device=DEV)
    with pytest.raises(hx.HelmError):  # 2D grids use the 7-point stencil
        hx.helm_apply(hx.Grid(n=(1, 20, 20), h=10.0, npml=3, v_ref=2000.0, stencil="27pt"), m_t, 1.0, x_t)
    m2 = torch.ones((2, 20, 20), dtype=torch.float32, device=DEV) * 1e-7
    x2 = torch.zeros((2, 20, 20), dtype=torch.complex64, device=DEV)
    with pytest.raises(hx.HelmError):  # a first axis of two nodes is neither 2D nor 3D
        hx.helm_apply(hx.Grid(n=(2, 20, 20), h=10.0, npml=0, v_ref=2000.0), m2, 1.0, x2)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_2d_noalloc_matches_apply(dtype):
    """helm_apply_noalloc on 2D grids, two calls in a row (the second
    smaller), against helm_apply and the oracle's 2D assembly."""
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    rdt = torch.float32 if dtype == "c64" else torch.float64
    tol = 1e-5 if dtype == "c64" else 1e-12
    for k, (n, npml, nrhs) in enumerate((((90, 64), 6, 3), ((40, 30), 3, 2))):
        print(f"case 2d noalloc {dtype} call {k} n={n}", flush=True)
        rng, m, vref, omega, h = _case(n, npml, seed=91 + k)
        grid = hx.Grid(n=(1,) + n, h=h, npml=npml, v_ref=vref, dtype=dtype)
        m_t = torch.tensor(m, dtype=rdt, device=DEV)
        x_t = torch.tensor(rng.standard_normal((nrhs, 1) + n) + 1j * rng.standard_normal((nrhs, 1) + n), dtype=cdt,
                           device=DEV)
        y_ref = hx.helm_apply(grid, m_t, omega, x_t)
        y_na = torch.full_like(x_t, float("nan"))
        hx.helm_apply_noalloc(grid, m_t, omega, x_t, y_na)
        torch.cuda.synchronize()
        a = y_na.cpu().numpy().astype(np.complex128)
        b = y_ref.cpu().numpy().astype(np.complex128)
        assert np.all(np.isfinite(a)) and np.linalg.norm(a - b) <= tol * np.linalg.norm(b)
        g = ops.make_grid((1,) + n, h, npml, omega, vref)
        H = m25.assemble2d(g, m_t.cpu().numpy().astype(np.float64), 0.0)
        ref = H @ x_t[-1].cpu().numpy().astype(np.complex128).ravel()
        assert np.linalg.norm(a[-1].ravel() - ref) <= tol * np.linalg.norm(ref)
