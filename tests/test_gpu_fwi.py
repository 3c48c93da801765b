"""GPU parity of misfit_gradient and the HelmholtzMisfit autograd Function
against the FP64 oracle (misfit, adjoint-state gradient), the zero-residual
special case, and central finite differences of the oracle."""
import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import operators as ops
from oracle import fwi

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _problem(stencil="7pt", seed=30, n=(28, 26, 30), npml=5, dtype="c64"):
    w = workloads.layered_random_workload(n, 25.0, npml, 6.0, nsrc_xy=(2, 2),
                                          nrec_xy=(5, 4), seed=seed)
    w.stencil = stencil
    w.w27 = workloads.W27_DEFAULT if stencil == "27pt" else w.w27
    rdt = torch.float32 if dtype == "c64" else torch.float64
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    m_t = torch.tensor(w.m, dtype=rdt, device=DEV)
    m_used = m_t.cpu().numpy().astype(np.float64)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil=stencil, dtype=dtype,
                   w27=w.w27)
    # observed data from a perturbed model through the oracle (never the GPU)
    rng = np.random.default_rng(seed)
    m_true = m_used * (1.0 + 0.05 * rng.standard_normal(w.n) * (np.arange(w.n[2]) > 12))
    solve_t = fwi.LUSolver(g, m_true, stencil, w.w27)
    d = np.stack([fwi.sample(solve_t(fwi.point_source(g, p)), w.rec) for p in w.src])
    d_used = torch.tensor(d, dtype=cdt, device=DEV)
    return w, g, grid, m_t, m_used, d_used


@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_misfit_gradient_matches_oracle(stencil):
    print(f"case misfit_gradient {stencil}", flush=True)
    w, g, grid, m_t, m_used, d_t = _problem(stencil)
    opts = hx.SolverOpts(tol=1e-10, max_cycles=100)
    f, grad, infos = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, opts=opts)
    assert all(i.status == 0 for i in infos) and len(infos) == 2 * len(w.src)
    d = d_t.cpu().numpy().astype(np.complex128)
    f_o, g_o, _, _ = fwi.misfit_gradient(g, m_used, w.src, w.rec, d, stencil=stencil,
                                         w27=w.w27)
    assert abs(f - f_o) <= 1e-5 * abs(f_o)
    gg = grad.double().cpu().numpy()
    assert np.linalg.norm(gg - g_o) <= 1e-4 * np.linalg.norm(g_o)
    # per cell on random interior cells, with a floor of 1e-3 max|g|
    rng = np.random.default_rng(1)
    lo, hi = g.npml + 1, np.array(g.n) - g.npml - 1
    for _ in range(32):
        k = tuple(rng.integers(lo, hi[a]) for a in range(3))
        assert abs(gg[k] - g_o[k]) <= 1e-4 * max(abs(g_o[k]), 1e-3 * np.abs(g_o).max())


def test_gradient_vs_exact_central_difference():
    """GPU gradient vs the oracle's exact central FD (eps = 1e-3 m_k) on 32
    random interior cells.  The solves run to 1e-10 (FP64 outer refinement)
    so that the per-cell comparison is not limited by the solve tolerance in
    low-amplitude cells."""
    w, g, grid, m_t, m_used, d_t = _problem(seed=31)
    f, grad, _ = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t,
                                    opts=hx.SolverOpts(tol=1e-10, max_cycles=100))
    gg = grad.double().cpu().numpy()
    d = d_t.cpu().numpy().astype(np.complex128)
    solve = fwi.LUSolver(g, m_used)
    us = [solve(fwi.point_source(g, p)) for p in w.src]
    _, rs = fwi.misfit(us, d, w.rec)
    rng = np.random.default_rng(2)
    lo, hi = g.npml + 1, np.array(g.n) - g.npml - 1
    gmax = np.abs(gg).max()
    for _ in range(32):
        k = tuple(rng.integers(lo, hi[a]) for a in range(3))
        fd = fwi.exact_central_difference(g, m_used, k, 1e-3 * m_used[k], us, rs, w.rec, solve)
        assert abs(gg[k] - fd) <= 1e-4 * max(abs(fd), 1e-3 * gmax)


def test_zero_residual_gives_zero_gradient():
    """d = P_r u(m) computed by the oracle (complex128, so the data carry no
    rounding of their own): f and g vanish up to the solve tolerance, far
    below their values for the perturbed-model data of the same problem."""
    w, g, grid, m_t, m_used, d_pert = _problem(seed=32, dtype="c128")
    solve = fwi.LUSolver(g, m_used)
    d = np.stack([fwi.sample(solve(fwi.point_source(g, p)), w.rec) for p in w.src])
    d_t = torch.tensor(d, dtype=torch.complex128, device=DEV)
    opts = hx.SolverOpts(tol=1e-12, max_cycles=120)
    f, grad, _ = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, opts=opts)
    fp, gp, _ = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_pert, opts=opts)
    print(f"zero residual: f {f:.3e} (perturbed {fp:.3e}); |g| {torch.linalg.norm(grad).item():.3e} "
          f"(perturbed {torch.linalg.norm(gp).item():.3e})", flush=True)
    assert f <= 1e-18 * 0.5 * np.sum(np.abs(d) ** 2)
    assert torch.linalg.norm(grad).item() <= 1e-6 * torch.linalg.norm(gp).item()


def test_autograd_function_matches_misfit_gradient():
    w, g, grid, m_t, m_used, d_t = _problem(seed=33)
    opts = hx.SolverOpts(tol=1e-10, max_cycles=100)
    m_req = m_t.clone().requires_grad_(True)
    f = hx.helmholtz_misfit(m_req, grid, w.omega, w.src, w.rec, d_t, opts)
    (2.0 * f).backward()
    f2, g2, _ = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, opts=opts)
    assert abs(float(f) - f2) <= 1e-6 * abs(f2)
    torch.testing.assert_close(m_req.grad, 2.0 * g2, rtol=1e-5, atol=1e-6 * g2.abs().max().item())


def test_accumulate_and_forward_only_flags():
    w, g, grid, m_t, m_used, d_t = _problem(seed=34)
    opts = hx.SolverOpts(tol=1e-10, max_cycles=100)
    f, g1, _ = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, opts=opts)
    g2 = g1.clone()
    f2, g2, _ = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, grad=g2,
                                   accumulate=True, opts=opts)
    torch.testing.assert_close(g2, 2 * g1, rtol=1e-5, atol=0.0)
    f3, none, infos = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t,
                                         forward_only=True, opts=opts)
    assert none is None and len(infos) == len(w.src)
    assert abs(f3 - f) <= 1e-6 * f
    with pytest.raises(hx.HelmError):
        bad = np.array(w.rec)
        bad[0, 0] = w.n[0]
        hx.misfit_gradient(grid, m_t, w.omega, w.src, bad, d_t, opts=opts)
    # the per-pair kernels index pairs by the second grid dimension: 65536
    # (frequency, source) pairs are refused before any device work
    many = np.repeat(np.asarray(w.src)[:1], 65536, axis=0)
    d_many = torch.zeros((1, 65536, len(w.rec)), dtype=d_t.dtype, device=DEV)
    with pytest.raises(hx.HelmError, match="65535"):
        hx.misfit_gradient(grid, m_t, w.omega, many, w.rec, d_many, opts=opts)


@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_multifrequency_masked_pairs_match_oracle(stencil):
    """Two frequencies x four sources in one call: complex amplitudes, a
    source/frequency mask (three pairs left out) and the average over the
    selected pairs; f, g and the stored fields of the selected pairs match
    the oracle's pair sum, unselected rows of the field store stay as they
    were, and the info entries of unselected pairs are zero."""
    print(f"case multifrequency {stencil}", flush=True)
    w, g, grid, m_t, m_used, _ = _problem(stencil, seed=35)
    rng = np.random.default_rng(35)
    omegas = [w.omega, 1.3 * w.omega]
    ns, nr = len(w.src), len(w.rec)
    d = (rng.standard_normal((2, ns, nr)) + 1j * rng.standard_normal((2, ns, nr))) * 1e-5
    amp = rng.standard_normal((2, ns)) + 1j * rng.standard_normal((2, ns))
    mask = np.array([[True, False, True, True], [False, True, True, False]])
    d_t = torch.tensor(d, dtype=torch.complex64, device=DEV)
    d_used = d_t.cpu().numpy().astype(np.complex128)
    store = torch.full((2, ns) + tuple(w.n), 7.0, dtype=torch.complex128, device=DEV)
    opts = hx.SolverOpts(tol=1e-10, max_cycles=100)
    f, grad, infos = hx.misfit_gradient(grid, m_t, omegas, w.src, w.rec, d_t, src_amp=amp, mask=mask,
                                        u_store=store, u_fp64=True, renormalise=True, opts=opts)
    f_o, g_o, us, _ = fwi.misfit_gradient_pairs(g, m_used, omegas, w.src, w.rec, d_used, amp=amp,
                                                mask=mask, renormalise=True, stencil=stencil, w27=w.w27)
    print(f"  f {f:.9e} oracle {f_o:.9e}", flush=True)
    assert len(infos) == 2 * 2 * ns
    for k, sel in enumerate(mask.ravel()):
        for inf in (infos[k], infos[2 * ns + k]):
            if sel:
                assert inf.status == 0 and inf.cycles >= 1
            else:
                assert inf.cycles == 0 and inf.matvecs == 0
    assert abs(f - f_o) <= 1e-5 * abs(f_o)
    gg = grad.double().cpu().numpy()
    assert np.linalg.norm(gg - g_o) <= 1e-4 * np.linalg.norm(g_o)
    st = store.cpu().numpy()
    for fi in range(2):
        for s in range(ns):
            if mask[fi, s]:
                u = us[(fi, s)]
                assert np.linalg.norm(st[fi, s] - u) <= 1e-6 * np.linalg.norm(u)
            else:
                assert np.all(st[fi, s] == 7.0)
    # the same selection through the autograd Function
    m_req = m_t.clone().requires_grad_(True)
    fa = hx.helmholtz_misfit(m_req, grid, omegas, w.src, w.rec, d_t, opts, src_amp=amp, mask=mask,
                             renormalise=True)
    fa.backward()
    assert abs(float(fa.detach()) - f) <= 1e-6 * abs(f)
    torch.testing.assert_close(m_req.grad, grad, rtol=1e-5, atol=1e-6 * grad.abs().max().item())


def test_two_frequency_call_equals_two_accumulated_calls():
    """One two-frequency call equals two one-frequency calls, the second
    accumulating into the gradient (the misfit is a sum over frequencies)."""
    w, g, grid, m_t, m_used, d_t = _problem(seed=36)
    opts = hx.SolverOpts(tol=1e-10, max_cycles=100)
    omegas = [w.omega, 0.8 * w.omega]
    d2 = torch.stack([d_t, 0.5 * d_t])
    f2, g2, _ = hx.misfit_gradient(grid, m_t, omegas, w.src, w.rec, d2, opts=opts)
    fa, ga, _ = hx.misfit_gradient(grid, m_t, omegas[0], w.src, w.rec, d2[0], opts=opts)
    fb, ga, _ = hx.misfit_gradient(grid, m_t, omegas[1], w.src, w.rec, d2[1], grad=ga, accumulate=True,
                                   opts=opts)
    assert abs(f2 - (fa + fb)) <= 1e-6 * abs(f2)
    torch.testing.assert_close(g2, ga, rtol=1e-4, atol=1e-5 * g2.abs().max().item())


@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_odd_nz_misfit_gradient_matches_oracle(stencil):
    """Odd z size: the fine level of the misfit solve keeps the caller's
    layout (one point per lane) under even-pitch pair-tiled coarse levels."""
    print(f"case odd nz misfit {stencil}", flush=True)
    w, g, grid, m_t, m_used, d_t = _problem(stencil, seed=37, n=(27, 25, 29))
    f, grad, infos = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t,
                                        opts=hx.SolverOpts(tol=1e-10, max_cycles=100))
    assert all(i.status == 0 for i in infos)
    d = d_t.cpu().numpy().astype(np.complex128)
    f_o, g_o, _, _ = fwi.misfit_gradient(g, m_used, w.src, w.rec, d, stencil=stencil, w27=w.w27)
    assert abs(f - f_o) <= 1e-5 * abs(f_o)
    gg = grad.double().cpu().numpy()
    assert np.linalg.norm(gg - g_o) <= 1e-4 * np.linalg.norm(g_o)
