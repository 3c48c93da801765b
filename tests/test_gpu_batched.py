"""GPU tests of the batched uneven solve: each member's result equals its own
plain solve (same kernels, same reduction order), matches the FP64 oracle's
exact solution at a tightened tolerance, is independent of the batch order,
and a diverging/zero member does not disturb the others."""
import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import operators as ops
from oracle import fwi

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _members(count=5, seed=40, lo=20, hi=34):
    params = workloads.c4_problem_params(count=count, seed=seed, lo=lo, hi=hi)
    out = []
    for p in params:
        w = workloads.c4_problem(p, sigma_cells=3.0)
        grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
        m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
        g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
        q = fwi.point_source(g, w.src[0])
        q_t = torch.tensor(q, dtype=torch.complex64, device=DEV)
        out.append((w, grid, m_t, q_t, g, q))
    return out


def test_batched_equals_plain_and_oracle():
    print("case batched 5 uneven members", flush=True)
    mem = _members()
    opts = hx.SolverOpts(tol=1e-8, max_cycles=60)
    us, infos = hx.helm_solve_batched([(b[1], b[2], b[0].omega, b[3]) for b in mem], opts=opts)
    for (w, grid, m_t, q_t, g, q), u_b, ib in zip(mem, us, infos):
        assert ib.status == 0 and ib.relres_fp64 <= 1e-8
        u_p, ip = hx.helm_solve(grid, m_t, w.omega, q_t, opts=opts)
        # same kernels; the stencil tiles (and so the order of partial sums)
        # may differ between the batch and the single problem, so the cycle
        # counts agree to within one and the results to the tolerance
        assert abs(ib.cycles - ip[0].cycles) <= 1
        d = torch.linalg.norm(u_b - u_p).item() / torch.linalg.norm(u_p).item()
        assert d <= 1e-6
        m_used = m_t.cpu().numpy().astype(np.float64)
        ue = fwi.LUSolver(g, m_used)(q)
        ub = u_b.cpu().numpy().astype(np.complex128)
        assert np.linalg.norm(ub - ue) <= 1e-5 * np.linalg.norm(ue)


def test_batch_order_does_not_change_results():
    mem = _members(count=4, seed=41)
    opts = hx.SolverOpts(tol=1e-7)
    us1, _ = hx.helm_solve_batched([(b[1], b[2], b[0].omega, b[3]) for b in mem], opts=opts)
    perm = [2, 0, 3, 1]
    us2, _ = hx.helm_solve_batched([(mem[i][1], mem[i][2], mem[i][0].omega, mem[i][3]) for i in perm],
                                   opts=opts)
    for k, i in enumerate(perm):
        assert torch.equal(us1[i], us2[k])


def test_batched_member_failure_is_isolated():
    mem = _members(count=3, seed=42)
    q_bad = mem[1][3].clone()
    q_bad[2, 2, 2] = float("nan")
    probs = [(mem[0][1], mem[0][2], mem[0][0].omega, mem[0][3]),
             (mem[1][1], mem[1][2], mem[1][0].omega, q_bad),
             (mem[2][1], mem[2][2], mem[2][0].omega, torch.zeros_like(mem[2][3]))]
    us, infos = hx.helm_solve_batched(probs, raise_on_failure=False)
    assert infos[0].status == 0 and infos[1].status == 2 and infos[2].status == 0
    assert torch.count_nonzero(us[2]).item() == 0
    w, grid, m_t, q_t, g, q = mem[0]
    r = q - ops.apply7(g, m_t.cpu().numpy().astype(np.float64), us[0].cpu().numpy().astype(np.complex128))
    assert np.linalg.norm(r) / np.linalg.norm(q) <= 2e-6


def test_batched_adjoint():
    mem = _members(count=3, seed=43)
    us, infos = hx.helm_solve_batched([(b[1], b[2], b[0].omega, b[3]) for b in mem], adjoint=True,
                                      opts=hx.SolverOpts(tol=1e-8, max_cycles=60))
    for (w, grid, m_t, q_t, g, q), u, inf in zip(mem, us, infos):
        assert inf.status == 0
        ue = fwi.LUSolver(g, m_t.cpu().numpy().astype(np.float64))(q, adjoint=True)
        assert np.linalg.norm(u.cpu().numpy() - ue) <= 1e-5 * np.linalg.norm(ue)


@pytest.mark.parametrize("adjoint", [False, True])
def test_batched_27pt_uneven_matches_oracle(adjoint):
    """Uneven compact 27-point members (even and odd nz, so different z
    pitches and staged tile sizes in one launch) against the oracle's exact
    solutions."""
    print(f"case batched 27-point uneven adjoint={adjoint}", flush=True)
    w27 = workloads.W27_DEFAULT
    rng = np.random.default_rng(44)
    shapes = [(22, 18, 26), (17, 24, 19), (20, 20, 31)]
    probs, refs = [], []
    for n in shapes:
        v = 1800.0 + 1200.0 * rng.random(n)
        m = 1.0 / v ** 2
        omega, h, npml = 2 * np.pi * 5.0, 20.0, 4
        grid = hx.Grid(n=n, h=h, npml=npml, v_ref=float(v.max()), stencil="27pt", dtype="c64", w27=w27)
        g = ops.make_grid(n, h, npml, omega, float(v.max()))
        m_t = torch.tensor(m, dtype=torch.float32, device=DEV)
        q = fwi.point_source(g, (n[0] // 2, n[1] // 2, n[2] // 2))
        q_t = torch.tensor(q, dtype=torch.complex64, device=DEV)
        probs.append((grid, m_t, omega, q_t))
        m_used = m_t.cpu().numpy().astype(np.float64)
        q_used = q_t.cpu().numpy().astype(np.complex128)
        refs.append(fwi.LUSolver(g, m_used, "27pt", w27)(q_used, adjoint=adjoint))
    us, infos = hx.helm_solve_batched(probs, adjoint=adjoint, opts=hx.SolverOpts(tol=1e-8, max_cycles=80))
    for u, info, ue in zip(us, infos, refs):
        assert info.status == 0 and info.relres_fp64 <= 1e-8
        ub = u.cpu().numpy().astype(np.complex128)
        assert np.linalg.norm(ub - ue) <= 1e-5 * np.linalg.norm(ue)
