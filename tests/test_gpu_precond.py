"""GPU parity of the ML-GMRES preconditioner itself (ML-GMRES section:
algorithm "Standard multigrid V-cycle" with GMRES smoothers, restriction,
recursive coarse FGMRES, prolongation) against the oracle, not only through
the converged solution:

* one outer FGMRES cycle from x = 0 (restart 5), and one single
  preconditioned step (restart 1: x = y M(q/||q||), the V-cycle's output up
  to the least-squares scalar), compared element by element with the
  oracle's iterate -- complex128 to 1e-10, complex64 (inner work in complex64,
  FP64 outer iterate) to 1e-4 -- for the 7-point and compact 27-point
  operators, forward and adjoint, on a ragged grid with odd sizes;
* the relative residual after each of the first three outer cycles against
  the oracle's (complex128);
* the number of outer cycles to 1e-6 against the oracle's count on the same
  inputs (tests/golden/precond_cycles.json, written by the oracle), within
  one cycle, including the constant-velocity 57^3 row of the paper's
  preconditioner table (n_lambda = 5, 8 points per wavelength).
A wrong restriction scale, a dropped smoothing step or a mis-ordered
recursion changes the one-cycle iterate far beyond these bounds."""
import json
import os

import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import operators as ops
from oracle import fwi, mlgmres

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precond_cycles.json")


def _case(stencil, dtype, n=(29, 27, 35), seed=50):
    w = workloads.layered_random_workload(n, 20.0, 5, 6.0, nsrc_xy=(2, 1), seed=seed)
    if stencil == "27pt":
        w.stencil, w.w27 = "27pt", workloads.W27_DEFAULT
    rdt = torch.float32 if dtype == "c64" else torch.float64
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    m_t = torch.tensor(w.m, dtype=rdt, device=DEV)
    m_used = m_t.cpu().numpy().astype(np.float64)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype=dtype, stencil=stencil, w27=w.w27)
    q_t = torch.tensor(np.stack([fwi.point_source(g, p) for p in w.src]), dtype=cdt, device=DEV)
    q_used = q_t.cpu().numpy().astype(np.complex128)
    return w, g, grid, m_t, m_used, q_t, q_used


@pytest.mark.parametrize("dtype,bar", [("c128", 1e-10), ("c64", 1e-4)])
@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("restart", [5, 1])
def test_one_outer_cycle_matches_oracle(stencil, dtype, bar, adjoint, restart):
    print(f"case one cycle {stencil} {dtype} adj={adjoint} restart={restart}", flush=True)
    w, g, grid, m_t, m_used, q_t, q_used = _case(stencil, dtype)
    opts = hx.SolverOpts(restart=restart, max_cycles=1, tol=1e-30)
    u_t, info = hx.helm_solve(grid, m_t, w.omega, q_t, adjoint=adjoint, opts=opts, raise_on_failure=False)
    u = u_t.cpu().numpy().astype(np.complex128)
    o = mlgmres.MLOptions(k_outer=restart)
    for s in range(len(w.src)):
        assert info[s].status == 1 and info[s].cycles == 1
        x, oi = mlgmres.mlgmres_solve(g, m_used, q_used[s], tol=1e-30, max_cycles=1, opts=o,
                                      stencil=stencil, w27=w.w27, adjoint=adjoint)
        err = np.linalg.norm(u[s] - x) / np.linalg.norm(x)
        print(f"  source {s}: |u - oracle| / |oracle| = {err:.3e}; relres gpu {info[s].relres_fp64:.6e} "
              f"oracle {oi['relres']:.6e}", flush=True)
        assert err <= bar
        assert abs(info[s].relres_fp64 - oi["relres"]) <= 10 * bar * oi["relres"] + 1e-12


@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_residual_history_matches_oracle_c128(stencil):
    """Relative residual of the outer iterate after 1, 2 and 3 cycles."""
    print(f"case residual history {stencil}", flush=True)
    w, g, grid, m_t, m_used, q_t, q_used = _case(stencil, "c128", n=(27, 31, 25), seed=51)
    hist = []
    mlgmres.mlgmres_solve(g, m_used, q_used[0], tol=1e-30, max_cycles=3, stencil=stencil, w27=w.w27,
                          history=hist)
    for k in (1, 2, 3):
        _, info = hx.helm_solve(grid, m_t, w.omega, q_t[:1], opts=hx.SolverOpts(max_cycles=k, tol=1e-30),
                                raise_on_failure=False)
        print(f"  after {k} cycles: gpu {info[0].relres_fp64:.9e} oracle {hist[k]:.9e}", flush=True)
        assert abs(info[0].relres_fp64 - hist[k]) <= 1e-8 * hist[k]


def _golden_cases():
    with open(GOLDEN) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_outer_cycle_counts_match_oracle(case):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_precond_cycles", os.path.join(os.path.dirname(GOLDEN), "make_precond_cycles.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    print(f"case cycle count {case['name']}", flush=True)
    w = mk.case_inputs(case)
    assert list(w.n) == case["grid"]
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64", stencil=w.stencil, w27=w.w27)
    m_t = torch.tensor(w.m, dtype=torch.float32, device=DEV)
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    q_t = torch.tensor(fwi.point_source(g, tuple(w.src[0])), dtype=torch.complex64, device=DEV)[None]
    _, info = hx.helm_solve(grid, m_t, w.omega, q_t, adjoint=case["adjoint"],
                            opts=hx.SolverOpts(tol=1e-6, max_cycles=30))
    print(f"  gpu cycles {info[0].cycles} (relres {info[0].relres_fp64:.3e}), oracle {case['oracle_cycles']}",
          flush=True)
    assert info[0].status == 0 and info[0].relres_fp64 <= 1e-6
    assert abs(info[0].cycles - case["oracle_cycles"]) <= 1
