"""GPU parity of the WRI (penalty method) objective, gradient and fields
(wri_misfit_gradient: receiver-space CG around batched ML-GMRES solves)
against the oracle's direct solve of the normal equations, over masked
(frequency, source) pairs with complex amplitudes and 1/#pairs, 7-point and
27-point, complex128 and complex64; the CG-free case (the reduced field);
and the argument checks."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import fwi, wri
from oracle import operators as ops

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
OMEGAS = (2 * np.pi * 5.0, 2 * np.pi * 6.5)
MASK = np.array([[True, False, True, True], [True, True, False, True]])


def _problem(stencil="7pt", dtype="c128", seed=130):
    n, npml = (16, 15, 14), 3
    w = workloads.layered_random_workload(n, 25.0, npml, 6.0, nsrc_xy=(2, 2), nrec_xy=(4, 4), seed=seed)
    w27 = workloads.W27_DEFAULT if stencil == "27pt" else (1, 0, 0, 1, 0, 0, 0)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    rdt = torch.float32 if dtype == "c64" else torch.float64
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    m_t = torch.tensor(w.m, dtype=rdt, device=DEV)
    m = m_t.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(seed)
    # data of a perturbed model plus noise, so the data and penalty terms both matter
    m_true = m * (1.0 + 0.05 * workloads.gaussian_random_field(rng, g.n, 2.0))
    d = np.zeros((2, 4, 16), np.complex128)
    for fi, om in enumerate(OMEGAS):
        from dataclasses import replace
        solve = fwi.LUSolver(replace(g, omega=om), m_true, stencil, w27 if stencil == "27pt" else None)
        for s in range(4):
            d[fi, s] = fwi.sample(solve(fwi.point_source(g, w.src[s])), w.rec)
    d += 0.05 * np.abs(d).mean() * (rng.standard_normal(d.shape) + 1j * rng.standard_normal(d.shape))
    d_t = torch.tensor(d, dtype=cdt, device=DEV)
    amp = rng.standard_normal((2, 4)) + 1j * rng.standard_normal((2, 4))
    H = ops.assemble(g, m, stencil, w27 if stencil == "27pt" else None)
    smax = float(spla.svds(H, k=1, return_singular_vectors=False, tol=1e-4)[0])
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil=stencil, dtype=dtype, w27=w27)
    return dict(w=w, g=g, grid=grid, m_t=m_t, m=m, d_t=d_t, d=d_t.cpu().numpy().astype(np.complex128), amp=amp,
                lam=3.0 / smax, w27=w27 if stencil == "27pt" else None, stencil=stencil)


# Bars.  complex128 with ML-GMRES to 1e-12 and the CG to 1e-10: the CG
# solves a receiver-space system whose condition number is about 1 +
# |P_r H^-1|^2 / lambda^2 (about 110 here), and its matrix-vector products carry
# the solves' 1e-12, so the field is good to ~1e-8 and f, g to ~1e-7.
# complex64: the solves' fields carry ~1e-6 relative error (FP32 inner work),
# amplified likewise: f 1e-3, g 1e-2.
@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
@pytest.mark.parametrize("dtype,tol,cg_tol,bf,bg,bu", [("c128", 1e-12, 1e-10, 1e-7, 1e-6, 1e-7),
                                                       ("c64", 1e-7, 1e-6, 1e-3, 1e-2, 1e-3)])
def test_wri_matches_oracle(stencil, dtype, tol, cg_tol, bf, bg, bu):
    print(f"case wri {stencil} {dtype}", flush=True)
    P = _problem(stencil, dtype)
    w = P["w"]
    u_store = torch.zeros((2, 4) + tuple(w.n), dtype=torch.complex128, device=DEV)
    f, grad, infos = hx.wri_misfit_gradient(P["grid"], P["m_t"], OMEGAS, w.src, w.rec, P["d_t"], P["lam"],
                                            src_amp=P["amp"], mask=MASK, renormalise=True, u_store=u_store,
                                            u_fp64=True, cg_tol=cg_tol, cg_max=100,
                                            opts=hx.SolverOpts(tol=tol, max_cycles=400))
    torch.cuda.synchronize()
    f_o, g_o, us_o = wri.wri_misfit_gradient_pairs(P["g"], P["m"], OMEGAS, w.src, w.rec, P["d"], P["lam"],
                                                   amp=P["amp"], mask=MASK, renormalise=True,
                                                   stencil=P["stencil"], w27=P["w27"])
    steps = [i.cycles for k, i in enumerate(infos) if MASK.ravel()[k]]
    eu = max(np.linalg.norm(u_store[fi, s].cpu().numpy() - us_o[(fi, s)]) / np.linalg.norm(us_o[(fi, s)])
             for fi in range(2) for s in range(4) if MASK[fi, s])
    ef = abs(f - f_o) / abs(f_o)
    eg = np.linalg.norm(grad.double().cpu().numpy() - g_o) / np.linalg.norm(g_o)
    print(f"  CG steps {steps}; field {eu:.2e}, f {ef:.2e}, g {eg:.2e}", flush=True)
    # every selected pair's CG reached cg_tol (CG in finite precision may take
    # more than nrec = 16 steps; the bound for condition ~110 is about 130)
    assert all(i.status == 0 for i in infos) and min(steps) >= 1
    assert eu <= bu and ef <= bf and eg <= bg
    for fi in range(2):
        for s in range(4):
            if not MASK[fi, s]:
                assert infos[fi * 4 + s].cycles == 0
                assert torch.count_nonzero(u_store[fi, s]) == 0


def test_wri_without_cg_steps_is_the_reduced_field():
    """cg_max = 0: u = H^{-1} q, so f = the reduced misfit (plus lambda^2/2
    times the solves' tiny residual) and the field equals misfit_gradient's."""
    P = _problem("7pt", "c128", seed=131)
    w = P["w"]
    opts = hx.SolverOpts(tol=1e-12, max_cycles=400)
    u1 = torch.zeros((2, 4) + tuple(w.n), dtype=torch.complex128, device=DEV)
    u2 = torch.zeros_like(u1)
    f, _, infos = hx.wri_misfit_gradient(P["grid"], P["m_t"], OMEGAS, w.src, w.rec, P["d_t"], P["lam"], mask=MASK,
                                         u_store=u1, cg_max=0, opts=opts, raise_on_failure=False)
    f_red, _, _ = hx.misfit_gradient(P["grid"], P["m_t"], OMEGAS, w.src, w.rec, P["d_t"], mask=MASK, u_store=u2,
                                     opts=opts)
    torch.cuda.synchronize()
    assert all(i.cycles == 0 for i in infos)
    assert abs(f - f_red) <= 1e-9 * f_red
    assert torch.allclose(u1, u2, rtol=0, atol=1e-12 * float(u2.abs().max()))


def test_wri_argument_checks():
    P = _problem("7pt", "c128", seed=132)
    w = P["w"]
    args = (P["grid"], P["m_t"], OMEGAS, w.src, w.rec, P["d_t"])
    with pytest.raises(hx.HelmError):
        hx.wri_misfit_gradient(*args, 0.0)
    with pytest.raises(hx.HelmError):
        hx.wri_misfit_gradient(*args, P["lam"], cg_tol=1.5)
    with pytest.raises(ValueError):
        hx.wri_misfit_gradient(*args, P["lam"], u_fp64=True)
