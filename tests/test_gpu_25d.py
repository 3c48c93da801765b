"""GPU parity of 2.5D modelling, misfit and gradient (misfit_gradient_25d:
every (frequency, source, k_y) 2D problem in one batched solve per direction)
against the oracle's LU-based 2.5D module: the modelled data element by
element, the misfit and the gradient, over masked (frequency, source) pairs
with complex amplitudes, 1/#pairs and sources and receivers at their own
coordinates along the invariant axis; modelling without data; argument
checks."""
import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
from oracle import model25d as m25
from oracle import operators as ops

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
OMEGAS = (2 * np.pi * 5.0, 2 * np.pi * 7.0)
MASK = np.array([[True, False, True], [True, True, True]])
NKY, PKC, VMIN = 12, 1.5, 1600.0


def _problem(dtype, seed=140, n2=44):
    rng = np.random.default_rng(seed)
    n1, h, npml = 60, 20.0, 6
    depth = np.linspace(0, 1, n2)
    v = (1600.0 + 1400.0 * depth)[None, None, :] * (1 + 0.04 * rng.standard_normal((1, n1, n2)))
    v = np.maximum(v, VMIN)
    rdt = torch.float32 if dtype == "c64" else torch.float64
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    m_t = torch.tensor(1.0 / v ** 2, dtype=rdt, device=DEV)
    g = ops.make_grid((1, n1, n2), h, npml, 1.0, float(v.max()))
    src = np.array([(15, 8), (30, 9), (45, 8)])
    src_y = np.array([0.0, 35.0, -20.0])
    rec = np.array([(j, 12) for j in range(8, 52, 4)])
    rec_y = np.linspace(-150.0, 200.0, len(rec))
    amp = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    d = (rng.standard_normal((2, 3, len(rec))) + 1j * rng.standard_normal((2, 3, len(rec)))) * 1e-3
    d_t = torch.tensor(d, dtype=cdt, device=DEV)
    grid = hx.Grid(n=(1, n1, n2), h=h, npml=npml, v_ref=float(v.max()), dtype=dtype)
    return dict(g=g, grid=grid, m_t=m_t, m=m_t.cpu().numpy().astype(np.float64), src=src, src_y=src_y, rec=rec,
                rec_y=rec_y, amp=amp, d_t=d_t, d=d_t.cpu().numpy().astype(np.complex128))


# complex128 with the solves at 1e-11: data and gradient to ~1e-9 of the
# oracle's exact solves; complex64 with FP32 inner work and the solves at
# 1e-7 (FP64 outer residual): the data and misfit as the 3D misfit tests
# (1e-5), the gradient, formed from the FP32 fields, to 1e-4.
# (an odd plane length keeps the fine level in the caller's layout: the
# one-point-per-lane operator there, pair tiles on the coarse levels)
@pytest.mark.parametrize("dtype,tol,bd,bf,bg,n2", [("c128", 1e-11, 1e-8, 1e-8, 1e-7, 44),
                                                   ("c64", 1e-7, 1e-5, 1e-5, 1e-4, 44),
                                                   ("c64", 1e-7, 1e-5, 1e-5, 1e-4, 43)])
def test_25d_matches_oracle(dtype, tol, bd, bf, bg, n2):
    print(f"case 2.5d {dtype} n2={n2}", flush=True)
    P = _problem(dtype, n2=n2)
    f, grad, d_pred, infos = hx.misfit_gradient_25d(P["grid"], P["m_t"], OMEGAS, P["src"], P["src_y"], P["rec"],
                                                    P["rec_y"], P["d_t"], nky=NKY, p_kc=PKC, v_min=VMIN,
                                                    src_amp=P["amp"], mask=MASK, renormalise=True,
                                                    opts=hx.SolverOpts(tol=tol, max_cycles=400))
    torch.cuda.synchronize()
    dp_o, f_o, g_o = m25.misfit_gradient_pairs(P["g"], P["m"], OMEGAS, P["src"], P["src_y"], P["rec"], P["rec_y"],
                                               P["d"], NKY, PKC, VMIN, amp=P["amp"], mask=MASK, renormalise=True)
    dp = d_pred.cpu().numpy().astype(np.complex128)
    ed = np.linalg.norm(dp[MASK] - dp_o[MASK]) / np.linalg.norm(dp_o[MASK])
    ef = abs(f - f_o) / f_o
    eg = np.linalg.norm(grad.double().cpu().numpy() - g_o) / np.linalg.norm(g_o)
    print(f"  data {ed:.2e}, misfit {ef:.2e}, gradient {eg:.2e}; cycles max "
          f"{max(i.cycles for i in infos)}", flush=True)
    assert np.all(dp[~MASK] == 0)
    assert ed <= bd and ef <= bf and eg <= bg
    # solves of unselected pairs did not run
    nfs = 2 * 3
    for k in range(nfs):
        if not MASK.ravel()[k]:
            assert all(infos[k * NKY + i].matvecs == 0 for i in range(NKY))


def test_25d_modelling_without_data():
    P = _problem("c64", seed=141)
    f, grad, d_pred, _ = hx.misfit_gradient_25d(P["grid"], P["m_t"], OMEGAS[0], P["src"], P["src_y"], P["rec"],
                                                P["rec_y"], None, nky=NKY, p_kc=PKC, v_min=VMIN,
                                                opts=hx.SolverOpts(tol=1e-7, max_cycles=200))
    torch.cuda.synchronize()
    dp_o, _, _ = m25.misfit_gradient_pairs(P["g"], P["m"], [OMEGAS[0]], P["src"], P["src_y"], P["rec"], P["rec_y"],
                                           None, NKY, PKC, VMIN)
    dp = d_pred.cpu().numpy().astype(np.complex128)
    assert grad is None
    assert np.linalg.norm(dp - dp_o) <= 1e-5 * np.linalg.norm(dp_o)
    assert abs(f - 0.5 * float(np.sum(np.abs(dp_o) ** 2))) <= 1e-5 * f


def test_25d_argument_checks():
    P = _problem("c64", seed=142)
    args = (P["m_t"], OMEGAS, P["src"], P["src_y"], P["rec"], P["rec_y"], P["d_t"])
    with pytest.raises(hx.HelmError):
        hx.misfit_gradient_25d(P["grid"], *args, nky=0)
    with pytest.raises(hx.HelmError):
        hx.misfit_gradient_25d(P["grid"], *args, v_min=0.0)
    bad = P["rec"].copy()
    bad[2, 1] = P["grid"].n[2]
    with pytest.raises(hx.HelmError):
        hx.misfit_gradient_25d(P["grid"], P["m_t"], OMEGAS, P["src"], P["src_y"], bad, P["rec_y"], P["d_t"])
    g3 = hx.Grid(n=(3,) + tuple(P["grid"].n[1:]), h=20.0, npml=1, v_ref=3000.0)
    m3 = torch.ones(tuple(g3.n), dtype=torch.float32, device=DEV) * 1e-7
    with pytest.raises(hx.HelmError):
        hx.misfit_gradient_25d(g3, m3, OMEGAS, P["src"], P["src_y"], P["rec"], P["rec_y"], P["d_t"])
    # 2 frequencies x 8 sources x 4096 nodes = 65536 2D problems: one more
    # than the second grid dimension of the per-problem kernels holds
    src8, y8 = np.repeat(P["src"][:1], 8, axis=0), np.zeros(8)
    d8 = torch.zeros((2, 8, len(P["rec"])), dtype=P["d_t"].dtype, device=DEV)
    with pytest.raises(hx.HelmError, match="65535"):
        hx.misfit_gradient_25d(P["grid"], P["m_t"], OMEGAS, src8, y8, P["rec"], P["rec_y"], d8, nky=4096)
