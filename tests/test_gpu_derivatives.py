"""GPU parity of pde_derivative (Jacobian, its adjoint, Gauss-Newton and full
Hessian products over (frequency, source) pairs; Table derivstuff, Appendix
A) against the FP64 oracle, element by element, for the 7-point and compact
27-point operators, complex64 and complex128; the adjoint identity <J x, y> =
<x, J^* y> and the Hessian's symmetry on the GPU (the paper's adjoint-test
table); reuse of stored forward fields."""
import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import derivatives as dv
from oracle import fwi
from oracle import operators as ops

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
OMEGAS = (2 * np.pi * 6.0, 2 * np.pi * 7.5)
MASK = np.array([[True, False, True, True], [False, True, True, False]])


def _problem(stencil="7pt", dtype="c64", seed=60, n=(26, 24, 30), npml=5):
    w = workloads.layered_random_workload(n, 25.0, npml, 6.0, nsrc_xy=(2, 2),
                                          nrec_xy=(5, 4), seed=seed)
    w27 = workloads.W27_DEFAULT if stencil == "27pt" else (1, 0, 0, 1, 0, 0, 0)
    rdt = torch.float32 if dtype == "c64" else torch.float64
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    m_t = torch.tensor(w.m, dtype=rdt, device=DEV)
    m_used = m_t.cpu().numpy().astype(np.float64)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil=stencil, dtype=dtype, w27=w27)
    rng = np.random.default_rng(seed)
    dm = workloads.gaussian_random_field(rng, g.n, 2.0) * m_used
    dm_t = torch.tensor(dm, dtype=rdt, device=DEV)
    dm_used = dm_t.cpu().numpy().astype(np.float64)
    ns, nr = len(w.src), len(w.rec)
    amp = rng.standard_normal((2, ns)) + 1j * rng.standard_normal((2, ns))
    d = (rng.standard_normal((2, ns, nr)) + 1j * rng.standard_normal((2, ns, nr))) * 1e-4
    d_t = torch.tensor(d, dtype=cdt, device=DEV)
    y = rng.standard_normal((2, ns, nr)) + 1j * rng.standard_normal((2, ns, nr))
    y_t = torch.tensor(y, dtype=cdt, device=DEV)
    return dict(w=w, g=g, grid=grid, w27=w27, m_t=m_t, m=m_used, dm_t=dm_t, dm=dm_used, amp=amp,
                d_t=d_t, d=d_t.cpu().numpy().astype(np.complex128), y_t=y_t,
                y=y_t.cpu().numpy().astype(np.complex128))


def _call(P, mode, inp, **kw):
    w = P["w"]
    tol = 1e-9 if P["grid"].dtype == "c64" else 1e-11
    out, infos = hx.pde_derivative(mode, P["grid"], P["m_t"], OMEGAS, w.src, w.rec, inp,
                                   d=P["d_t"] if mode == "hessian" else None, src_amp=P["amp"],
                                   mask=MASK, opts=hx.SolverOpts(tol=tol, max_cycles=200), **kw)
    torch.cuda.synchronize()
    for k, row in enumerate(infos):
        for fi in range(2):
            for s in range(len(w.src)):
                if MASK[fi, s]:
                    assert row[fi * len(w.src) + s].status == 0, (mode, k, fi, s)
                else:
                    assert row[fi * len(w.src) + s].cycles == 0
    return out


@pytest.mark.parametrize("dtype,bar", [("c64", 1e-5), ("c128", 1e-9)])
@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_jacobian_matches_oracle(stencil, dtype, bar):
    print(f"case jacobian {stencil} {dtype}", flush=True)
    P = _problem(stencil, dtype)
    w = P["w"]
    J = _call(P, "jacobian", P["dm_t"]).cpu().numpy().astype(np.complex128)
    ref = dv.jacobian_forward_pairs(P["g"], P["m"], OMEGAS, w.src, w.rec, P["dm"], amp=P["amp"], mask=MASK,
                                    stencil=stencil, w27=P["w27"])
    err = np.linalg.norm(J - ref) / np.linalg.norm(ref)
    print(f"  |J - oracle| / |oracle| = {err:.3e}", flush=True)
    assert err <= bar
    assert np.all(J[~MASK] == 0)


@pytest.mark.parametrize("dtype,bar", [("c64", 1e-4), ("c128", 1e-9)])
@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
@pytest.mark.parametrize("mode", ["jacobian_adjoint", "hessian_gn", "hessian"])
def test_model_space_products_match_oracle(mode, stencil, dtype, bar):
    print(f"case {mode} {stencil} {dtype}", flush=True)
    P = _problem(stencil, dtype, seed=61)
    w = P["w"]
    kw = dict(amp=P["amp"], mask=MASK, renormalise=True, stencil=stencil, w27=P["w27"])
    if mode == "jacobian_adjoint":
        out = _call(P, mode, P["y_t"], renormalise=True)
        ref = dv.jacobian_adjoint_pairs(P["g"], P["m"], OMEGAS, w.src, w.rec, P["y"], **kw)
    elif mode == "hessian_gn":
        out = _call(P, mode, P["dm_t"], renormalise=True)
        ref = dv.hessian_gn_pairs(P["g"], P["m"], OMEGAS, w.src, w.rec, P["dm"], **kw)
    else:
        out = _call(P, mode, P["dm_t"], renormalise=True)
        ref = dv.hessian_full_pairs(P["g"], P["m"], OMEGAS, w.src, w.rec, P["d"], P["dm"], **kw)
    o = out.double().cpu().numpy()
    err = np.linalg.norm(o - ref) / np.linalg.norm(ref)
    print(f"  |out - oracle| / |oracle| = {err:.3e}", flush=True)
    assert err <= bar
    # per cell on interior cells, floor 1e-3 max|ref|
    rng = np.random.default_rng(5)
    g = P["g"]
    lo, hi = g.npml + 1, np.array(g.n) - g.npml - 1
    for _ in range(32):
        k = tuple(rng.integers(lo, hi[a]) for a in range(3))
        assert abs(o[k] - ref[k]) <= 10 * bar * max(abs(ref[k]), 1e-3 * np.abs(ref).max())


@pytest.mark.parametrize("dtype,bar", [("c64", 1e-5), ("c128", 1e-10)])
@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_adjoint_identity_and_hessian_symmetry_on_gpu(stencil, dtype, bar):
    """<J x, y> = <x, J^* y> and <H x, z> = <x, H z> for the GPU products
    (the paper's adjoint-test table, Jacobian and Hessian rows)."""
    print(f"case adjoint identity {stencil} {dtype}", flush=True)
    P = _problem(stencil, dtype, seed=62)
    Jx = _call(P, "jacobian", P["dm_t"]).cpu().numpy().astype(np.complex128)
    Jty = _call(P, "jacobian_adjoint", P["y_t"]).double().cpu().numpy()
    a = float(np.real(np.vdot(P["y"], Jx)))
    b = float(np.sum(P["dm"] * Jty))
    print(f"  <Jx, y> = {a:.10e}  <x, J*y> = {b:.10e}", flush=True)
    assert abs(a - b) <= bar * np.linalg.norm(Jx) * np.linalg.norm(P["y"])
    rng = np.random.default_rng(9)
    z = workloads.gaussian_random_field(rng, P["g"].n, 2.0) * P["m"]
    z_t = torch.tensor(z, dtype=P["m_t"].dtype, device=DEV)
    z = z_t.cpu().numpy().astype(np.float64)
    Hx = _call(P, "hessian", P["dm_t"]).double().cpu().numpy()
    Hz = _call(P, "hessian", z_t).double().cpu().numpy()
    a, b = float(np.sum(Hx * z)), float(np.sum(P["dm"] * Hz))
    print(f"  <Hx, z> = {a:.10e}  <x, Hz> = {b:.10e}", flush=True)
    assert abs(a - b) <= 10 * bar * np.linalg.norm(Hx) * np.linalg.norm(z)


def test_reuse_of_stored_forward_fields():
    """Forward fields stored by misfit_gradient (FP64 iterates) and reused:
    the Gauss-Newton product equals the one that solves them again, and the
    forward-field info rows stay empty."""
    P = _problem("7pt", "c64", seed=63)
    w, grid = P["w"], P["grid"]
    ns = len(w.src)
    opts = hx.SolverOpts(tol=1e-9, max_cycles=200)
    u = torch.empty((2, ns) + tuple(w.n), dtype=torch.complex128, device=DEV)
    hx.misfit_gradient(grid, P["m_t"], OMEGAS, w.src, w.rec, P["d_t"], src_amp=P["amp"], mask=MASK,
                       u_store=u, u_fp64=True, forward_only=True, opts=opts)
    a, inf = hx.pde_derivative("hessian_gn", grid, P["m_t"], OMEGAS, w.src, w.rec, P["dm_t"], src_amp=P["amp"],
                               mask=MASK, u_store=u, reuse_u=True, u_fp64=True, opts=opts)
    assert all(i.cycles == 0 for i in inf[0])
    b = _call(P, "hessian_gn", P["dm_t"])
    torch.cuda.synchronize()
    a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)


def test_accumulate_and_rejections():
    P = _problem("7pt", "c64", seed=64)
    w, grid = P["w"], P["grid"]
    base = _call(P, "jacobian_adjoint", P["y_t"])
    acc = base.clone()
    _call(P, "jacobian_adjoint", P["y_t"], out=acc, accumulate=True)
    torch.cuda.synchronize()
    assert torch.allclose(acc, 2 * base, rtol=1e-5, atol=1e-5 * float(base.abs().max()))
    with pytest.raises(ValueError):
        hx.pde_derivative("hessian", grid, P["m_t"], OMEGAS, w.src, w.rec, P["dm_t"])  # no data
    with pytest.raises(hx.HelmError):
        hx.pde_derivative("jacobian", grid, P["m_t"], OMEGAS, w.src, np.array([[0, 0, 999]]), P["dm_t"])
