"""GPU parity at the full sizes of the workloads, in the launch
configurations bench.py times.  Where the oracle cannot solve at that size,
it checks what holds at any size: the FP64 residual of the returned fields,
recomputed on the CPU with the oracle's operator.  The operator itself is
compared array-wide at the largest (27-point) size."""
import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import operators as ops
from oracle import fwi

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _relres(g, m, u, q, stencil="7pt", w27=None, adjoint=False):
    r = q - ops.apply(g, m, u, adjoint=adjoint, stencil=stencil, w27=w27)
    return np.linalg.norm(r) / np.linalg.norm(q)


def test_c2_full_multisource_solve_is_certified():
    """128^3 layered model, all 16 sources in one multi-right-hand-side
    forward solve (as in the bench step): the FP64 fields returned satisfy
    ||q - H u|| / ||q|| <= 1e-6 with the residual recomputed by the oracle,
    and the GPU's own FP64 certificate agrees with the oracle's value."""
    print("case full c2 128^3 x 16 sources", flush=True)
    w = workloads.c2_layered()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
    m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
    rec = workloads.surface_positions(w.n, w.npml, (4, 4))
    nsrc = len(w.src)
    d = torch.zeros((nsrc, len(rec)), dtype=torch.complex64, device=DEV)
    u = torch.empty((nsrc,) + w.n, dtype=torch.complex128, device=DEV)
    _, _, infos = hx.misfit_gradient(grid, m_t, w.omega, w.src, rec, d, u_store=u, forward_only=True,
                                     u_fp64=True, opts=hx.SolverOpts(tol=1e-6, max_cycles=30))
    assert all(i.status == 0 and i.relres_fp64 <= 1e-6 for i in infos[:nsrc])
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    m_used = m_t.cpu().numpy().astype(np.float64)
    for s in (0, 7, 15):
        # the library injects the source in complex64: the oracle uses that value
        q = fwi.point_source(g, tuple(w.src[s])).astype(np.complex64).astype(np.complex128)
        rel = _relres(g, m_used, u[s].cpu().numpy(), q)
        assert rel <= 1e-6
        assert abs(rel - infos[s].relres_fp64) <= 1e-3 * rel


def test_c5_full_size_27pt_operator():
    """320x320x160 salt model, 27-point operator, 8 right-hand sides in one
    launch: forward (right-hand side 0) and adjoint (right-hand side 5) equal
    the oracle's FP64 evaluation over the whole array."""
    print("case full c5 320x320x160 27pt x 8", flush=True)
    w = workloads.c5_salt()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil="27pt", dtype="c64", w27=w.w27)
    m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
    gen = torch.Generator(device="cpu").manual_seed(5)
    x_t = torch.randn((8,) + w.n, dtype=torch.complex64, generator=gen).to(DEV)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    m_used = m_t.cpu().numpy().astype(np.float64)
    for adjoint, r in ((False, 0), (True, 5)):
        y_t = hx.helm_apply(grid, m_t, w.omega, x_t, adjoint=adjoint)
        torch.cuda.synchronize()
        y = y_t[r].cpu().numpy().astype(np.complex128)
        del y_t
        ref = ops.apply(g, m_used, x_t[r].cpu().numpy().astype(np.complex128), adjoint=adjoint,
                        stencil="27pt", w27=w.w27)
        assert np.linalg.norm(y - ref) <= 1e-5 * np.linalg.norm(ref)
        assert np.abs(y - ref).max() <= 4e-5 * np.abs(ref).max()


def test_c4_full_size_members_batched_and_plain():
    """The first six problems of the seeded 256-problem uneven draw (dims
    48-160) solved together and one at a time: every FP64 certificate <= 1e-6,
    and the returned complex64 fields solve the oracle's system (the residual
    recomputed in FP64 includes the rounding of the fields to complex64)."""
    print("case full c4 first 6 members", flush=True)
    params = workloads.c4_problem_params(count=256)[:6]
    probs, meta = [], []
    for p in params:
        w = workloads.c4_problem(p)
        grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
        m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
        g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
        q = fwi.point_source(g, tuple(w.src[0]))
        probs.append((grid, m_t, w.omega, torch.tensor(q, dtype=torch.complex64, device=DEV)))
        meta.append((g, q, m_t.cpu().numpy().astype(np.float64)))
    opts = hx.SolverOpts(tol=1e-6, max_cycles=40)
    ub, ib = hx.helm_solve_batched(probs, opts=opts)
    for k, (pr, (g, q, m_used)) in enumerate(zip(probs, meta)):
        up, ip = hx.helm_solve(*pr, opts=opts)
        assert ib[k].status == 0 and ib[k].relres_fp64 <= 1e-6
        assert ip[0].status == 0 and ip[0].relres_fp64 <= 1e-6
        for u in (ub[k], up):
            assert _relres(g, m_used, u.cpu().numpy().astype(np.complex128), q) <= 1e-4


def test_c5_full_27pt_solve_is_certified():
    """320x320x160 salt model, compact 27-point operator: two of the eight
    sources solved together (forward, FP64 fields returned) satisfy the
    oracle's FP64 residual ||q - H u|| / ||q|| <= 1e-6."""
    print("case full c5 320x320x160 27pt solve x 2", flush=True)
    w = workloads.c5_salt()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil="27pt", dtype="c64", w27=w.w27)
    m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
    src = w.src[[0, 5]]
    rec = w.rec[:16]
    d = torch.zeros((2, len(rec)), dtype=torch.complex64, device=DEV)
    u = torch.empty((2,) + w.n, dtype=torch.complex128, device=DEV)
    _, _, infos = hx.misfit_gradient(grid, m_t, w.omega, src, rec, d, u_store=u, forward_only=True, u_fp64=True,
                                     opts=hx.SolverOpts(tol=1e-6, max_cycles=30))
    assert all(i.status == 0 and i.relres_fp64 <= 1e-6 for i in infos[:2])
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    m_used = m_t.cpu().numpy().astype(np.float64)
    for s in range(2):
        # the library injects the source in complex64: the oracle uses that value
        q = fwi.point_source(g, tuple(src[s])).astype(np.complex64).astype(np.complex128)
        rel = _relres(g, m_used, u[s].cpu().numpy(), q, stencil="27pt", w27=w.w27)
        assert rel <= 1e-6
        assert abs(rel - infos[s].relres_fp64) <= 1e-3 * rel


def test_c3_full_fwi_gradient_directional_difference():
    """96^3 FWI configuration at full size (64 sources in one multi-source
    solve, 48x48 receivers, data from the true model, gradient at the
    smoothed start): sampled forward fields certified by the oracle's FP64
    residual, every solve converged, and the adjoint-state gradient against
    a central difference of the misfit along a smooth random direction dm,
    <g, dm> = (f(m + dm) - f(m - dm)) / 2, to 1e-3 relative.  The misfits
    come from tight GPU solves (FP64 iterates); the quotient's own error is
    of order |dm|^2."""
    from scipy import ndimage
    print("case full c3 96^3 x 64 sources gradient", flush=True)
    w = workloads.c3_fwi()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
    nsrc = len(w.src)
    tight = hx.SolverOpts(tol=1e-9, max_cycles=80)
    mt_t = torch.tensor(w.m_true, dtype=torch.float32, device=DEV)
    u = torch.empty((nsrc,) + w.n, dtype=torch.complex64, device=DEV)
    hx.misfit_gradient(grid, mt_t, w.omega, w.src, w.rec,
                       torch.zeros((nsrc, len(w.rec)), dtype=torch.complex64, device=DEV),
                       u_store=u, forward_only=True, opts=tight)
    ridx = torch.tensor(np.asarray(w.rec, np.int64), device=DEV)
    d_t = u[:, ridx[:, 0], ridx[:, 1], ridx[:, 2]].contiguous()
    del u, mt_t
    m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
    uf = torch.empty((nsrc,) + w.n, dtype=torch.complex128, device=DEV)
    f0, grad, infos = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, u_store=uf, u_fp64=True,
                                         opts=tight)
    assert len(infos) == 2 * nsrc and all(i.status == 0 and i.relres_fp64 <= 1e-9 for i in infos)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    m_used = m_t.cpu().numpy().astype(np.float64)
    for s in (0, 37, 63):
        q = fwi.point_source(g, tuple(w.src[s])).astype(np.complex64).astype(np.complex128)
        assert _relres(g, m_used, uf[s].cpu().numpy(), q) <= 2e-9
    del uf
    rng = np.random.default_rng(5)
    dm = ndimage.gaussian_filter(rng.standard_normal(w.n), 3.0)
    p = w.npml
    mask = np.zeros(w.n)
    mask[p:-p, p:-p, p:-p] = 1.0
    dm = dm * mask
    dm *= 1e-3 * m_used.min() / np.abs(dm).max()
    mp = torch.tensor(m_used + dm, dtype=torch.float32, device=DEV)
    mm = torch.tensor(m_used - dm, dtype=torch.float32, device=DEV)
    fp, _, ip = hx.misfit_gradient(grid, mp, w.omega, w.src, w.rec, d_t, forward_only=True, opts=tight)
    fm, _, im = hx.misfit_gradient(grid, mm, w.omega, w.src, w.rec, d_t, forward_only=True, opts=tight)
    assert all(i.status == 0 for i in ip + im)
    # the direction the GPU actually saw (both models rounded to float32)
    dm_used = (mp.cpu().numpy().astype(np.float64) - mm.cpu().numpy().astype(np.float64)) / 2
    lin = float(np.sum(grad.cpu().numpy().astype(np.float64) * dm_used))
    fd = (fp - fm) / 2
    print(f"c3 directional: <g,dm> = {lin:.6e}, central difference = {fd:.6e}", flush=True)
    assert abs(fd - lin) <= 1e-3 * abs(lin)


def test_c4_all_256_batched_sample_certified():
    """All 256 problems of the seeded uneven draw (3.2e8 points) in one
    batched solve, as bench.py times it: every FP64 certificate <= 1e-6, and
    a seeded sample of 8 returned fields solve the oracle's system (FP64
    residual recomputed on the CPU; it includes the rounding of the fields
    to complex64)."""
    import bench
    print("case full c4 all 256 batched", flush=True)
    params = workloads.c4_problem_params(count=256)
    members = bench.c4_members(params)
    probs = []
    for n, h, npml, vref, omega, src, m32 in members:
        grid = hx.Grid(n=n, h=h, npml=npml, v_ref=vref, dtype="c64")
        q_t = torch.zeros(n, dtype=torch.complex64, device=DEV)
        q_t[src] = 1.0 / h ** 3
        probs.append((grid, torch.from_numpy(m32).to(DEV), omega, q_t))
    ub, ib = hx.helm_solve_batched(probs, opts=hx.SolverOpts(tol=1e-6, max_cycles=40))
    assert all(i.status == 0 and i.relres_fp64 <= 1e-6 for i in ib)
    print(f"  all converged; mean cycles {np.mean([i.cycles for i in ib]):.2f}", flush=True)
    rng = np.random.default_rng(256)
    for k in sorted(rng.choice(256, size=8, replace=False)):
        n, h, npml, vref, omega, src, m32 = members[k]
        g = ops.make_grid(n, h, npml, omega, vref)
        q = probs[k][3].cpu().numpy().astype(np.complex128)
        rel = _relres(g, m32.astype(np.float64), ub[k].cpu().numpy().astype(np.complex128), q)
        print(f"  problem {k} {n}: GPU certificate {ib[k].relres_fp64:.3e}, oracle residual of the "
              f"complex64 field {rel:.3e}", flush=True)
        assert rel <= 1e-4


def test_c5_full_forward_adjoint_gradient():
    """320x320x160 salt model, compact 27-point operator, all 8 sources and
    300x300 receivers, data from the sharp model, misfit and gradient at the
    smoothed model: sampled forward fields (FP64 iterates) certified by the
    oracle's FP64 residual; the adjoint fields of two sources, solved from the
    adjoint sources -P_r^T r_s, certified with the oracle's adjoint operator;
    and <g, dm> against the central difference of the misfit along a smooth
    direction, to 1e-3 relative."""
    from scipy import ndimage
    print("case full c5 320x320x160 27pt forward + adjoint + gradient", flush=True)
    w = workloads.c5_salt()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil="27pt", dtype="c64", w27=w.w27)
    nsrc, nrec = len(w.src), len(w.rec)
    tight = hx.SolverOpts(tol=1e-8, max_cycles=60)
    mt_t = torch.tensor(w.m_true, dtype=torch.float32, device=DEV)
    u = torch.empty((nsrc,) + w.n, dtype=torch.complex64, device=DEV)
    hx.misfit_gradient(grid, mt_t, w.omega, w.src, w.rec, torch.zeros((nsrc, nrec), dtype=torch.complex64,
                                                                      device=DEV),
                       u_store=u, forward_only=True, opts=hx.SolverOpts(tol=1e-6, max_cycles=30))
    ridx = torch.tensor(np.asarray(w.rec, np.int64), device=DEV)
    d_t = u[:, ridx[:, 0], ridx[:, 1], ridx[:, 2]].contiguous()
    del u, mt_t
    torch.cuda.empty_cache()
    print("  data synthesised", flush=True)
    m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
    uf = torch.empty((nsrc,) + w.n, dtype=torch.complex128, device=DEV)
    f0, grad, infos = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, u_store=uf, u_fp64=True,
                                         opts=tight)
    assert len(infos) == 2 * nsrc and all(i.status == 0 and i.relres_fp64 <= 1e-8 for i in infos)
    print(f"  misfit {f0:.6e}; forward and adjoint solves converged", flush=True)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    m_used = m_t.cpu().numpy().astype(np.float64)
    d = d_t.cpu().numpy().astype(np.complex128)
    for s in (0, 6):
        us = uf[s].cpu().numpy()
        q = fwi.point_source(g, tuple(w.src[s])).astype(np.complex64).astype(np.complex128)
        rel = _relres(g, m_used, us, q, stencil="27pt", w27=w.w27)
        print(f"  forward field {s}: oracle residual {rel:.3e}", flush=True)
        assert rel <= 2e-8
        # adjoint source of this source's residual, solved on the GPU with H^H
        b = -fwi.sample_adjoint(g.n, w.rec, fwi.sample(us, w.rec) - d[s])
        b_t = torch.tensor(b, dtype=torch.complex64, device=DEV)[None]
        v_t, vi = hx.helm_solve(grid, m_t, w.omega, b_t, adjoint=True, opts=hx.SolverOpts(tol=1e-6, max_cycles=30))
        assert vi[0].status == 0 and vi[0].relres_fp64 <= 1e-6
        rel = _relres(g, m_used, v_t[0].cpu().numpy().astype(np.complex128),
                      b_t[0].cpu().numpy().astype(np.complex128), stencil="27pt", w27=w.w27, adjoint=True)
        print(f"  adjoint field {s}: GPU certificate {vi[0].relres_fp64:.3e}, oracle residual of the "
              f"complex64 field {rel:.3e}", flush=True)
        assert rel <= 1e-4
        del v_t
    del uf
    torch.cuda.empty_cache()
    rng = np.random.default_rng(6)
    dm = ndimage.gaussian_filter(rng.standard_normal(w.n), 4.0)
    p = w.npml
    mask = np.zeros(w.n)
    mask[p:-p, p:-p, p:-p] = 1.0
    dm = dm * mask
    dm *= 1e-3 * m_used.min() / np.abs(dm).max()
    mp = torch.tensor(m_used + dm, dtype=torch.float32, device=DEV)
    mm = torch.tensor(m_used - dm, dtype=torch.float32, device=DEV)
    fp, _, ip = hx.misfit_gradient(grid, mp, w.omega, w.src, w.rec, d_t, forward_only=True, opts=tight)
    fm, _, im = hx.misfit_gradient(grid, mm, w.omega, w.src, w.rec, d_t, forward_only=True, opts=tight)
    assert all(i.status == 0 for i in ip + im)
    dm_used = (mp.cpu().numpy().astype(np.float64) - mm.cpu().numpy().astype(np.float64)) / 2
    lin = float(np.sum(grad.cpu().numpy().astype(np.float64) * dm_used))
    fd = (fp - fm) / 2
    print(f"  c5 directional: <g,dm> = {lin:.6e}, central difference = {fd:.6e}", flush=True)
    assert abs(fd - lin) <= 1e-3 * abs(lin)
