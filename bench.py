#!/usr/bin/env python3
"""Benchmark of the MI355X Helmholtz hot path.

One step = one pass of the whole path over the 128^3 layered workload
(h = 12.5 m, 8 Hz, absorbing layer 15, velocity 1500-4500 m/s layers with 5 %
correlated perturbations, 16 sources on the top interior plane, 32 x 32
receivers): forward ML-GMRES solves of all 16 sources (complex64, FP64
residual, rel. res. 1e-6), receiver sampling and misfit, adjoint solves of
all 16 sources, and the gradient kernel -- misfit_gradient() through the C
ABI.  `value` = Helmholtz solves per second over the timed steps (32 solves
per step), inputs resident in HBM.

Also measured in the same run:
* the stencil kernel alone (helm_apply on the same grid with 16 right-hand
  sides) timed with HIP events on the launch stream, reported against the
  8 TB/s HBM peak with the algorithmic bytes 16*S + 4 per grid point, next
  to a plain device copy (the practical ceiling);
* the compact 27-point operator on the 320x320x160 salt workload (8
  right-hand sides), the same way;
* batched vs plain solves of uneven problems (helm_solve_batched vs
  helm_solve one at a time);
* on the 96^3 FWI workload: the linearised products (J, J^*, H_GN, full
  Hessian), off-grid sources and receivers, WRI and the inversion driver;
* the FP64 CPU oracle on a bounded sample of the same workload (rank 0).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
T_START = time.perf_counter()


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench {time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)
METRIC = ("stencil GB/s (% HBM peak) + Helmholtz solves/sec, batched vs plain, "
          "at rel.res 1e-6")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--stencil-reps", type=int, default=50)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--nrec", type=int, default=32, help="receivers per axis")
    p.add_argument("--batch-count", type=int, default=256,
                   help="problems of the uneven 256-problem draw used for batched vs plain")
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--stencil-only", action="store_true",
                   help="only the stencil measurement (for hardware-counter runs)")
    p.add_argument("--sweep", action="store_true",
                   help="only the stencil size sweep (7-point 64^3..512^3, 27-point), one JSON line per size")
    p.add_argument("--no-stencil27", action="store_true")
    p.add_argument("--no-c5", action="store_true",
                   help="skip the 320x320x160 27-point misfit + gradient evaluation (about 60 s)")
    p.add_argument("--c5-only", action="store_true")
    p.add_argument("--stencil27-only", action="store_true",
                   help="only the 27-point operator timing on the 320x320x160 workload (and a plain "
                        "copy of the same size, the calibration of hardware-counter runs)")
    p.add_argument("--batch-only", action="store_true", help="only batched vs plain")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the derivative / off-grid / WRI / driver timings on the 96^3 workload")
    p.add_argument("--extras-only", action="store_true")
    return p.parse_args()


def apply_timing(hx, torch, grid, m_t, omega, S, reps, dev):
    """Average helm_apply launch time (S right-hand sides, HIP events on the
    launch stream, two input/output pairs alternating) and its algorithmic
    GB/s ((16 S + 4) B per grid point)."""
    n = tuple(grid.n)
    xs = [torch.randn((S,) + n, dtype=torch.complex64, device=dev) for _ in range(2)]
    ys = [torch.empty_like(xs[0]) for _ in range(2)]
    for i in range(3):
        hx.helm_apply(grid, m_t, omega, xs[i % 2], out=ys[i % 2])
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(reps):
        hx.helm_apply(grid, m_t, omega, xs[i % 2], out=ys[i % 2])
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    npts = n[0] * n[1] * n[2]
    return ms, (16 * S + 4) * npts / (ms * 1e-3) / 1e9


def stencil27_timing(hx, torch, workloads, reps, dev):
    """The 27-point operator on the 320x320x160 salt workload, 8 right-hand
    sides (its sources), complex64."""
    w = workloads.c5_salt()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil="27pt", dtype="c64", w27=w.w27)
    m_t = torch.tensor(w.m, dtype=torch.float32, device=dev)
    ms, gbs = apply_timing(hx, torch, grid, m_t, w.omega, len(w.src), reps, dev)
    return {"kernel": "k_h27p<false,false,false> (helm_apply: complex64 compact 27-point, pair tiles, 8 rhs)",
            "workload": "320x320x160 salt model, h=15 m, 10 Hz", "ms_per_launch": round(ms, 5),
            "GB_s": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_point": "16*8+4"}


def c5_gradient(hx, torch, workloads, dev):
    """The 320x320x160 27-point salt case: one misfit + gradient evaluation
    (8 forward + 8 adjoint ML-GMRES solves to 1e-6 and the gradient) on the
    smoothed model, with observed data from the sharp model (synthesised
    first, untimed).  Timed warm (the first evaluation builds the solver)."""
    w = workloads.c5_salt()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, stencil="27pt", dtype="c64", w27=w.w27)
    opts = hx.SolverOpts(tol=1e-6, max_cycles=30)
    nsrc = len(w.src)
    mt_t = torch.tensor(w.m_true, dtype=torch.float32, device=dev)
    u = torch.empty((nsrc,) + w.n, dtype=torch.complex64, device=dev)
    hx.misfit_gradient(grid, mt_t, w.omega, w.src, w.rec,
                       torch.zeros((nsrc, len(w.rec)), dtype=torch.complex64, device=dev),
                       u_store=u, forward_only=True, opts=opts)
    ridx = torch.tensor(w.rec.astype(np.int64), device=dev)
    d_t = u[:, ridx[:, 0], ridx[:, 1], ridx[:, 2]].contiguous()
    del u, mt_t
    torch.cuda.empty_cache()
    m_t = torch.tensor(w.m, dtype=torch.float32, device=dev)
    grad = torch.empty(w.n, dtype=torch.float32, device=dev)
    # build the solver and capture its graphs (one outer cycle: same solver key)
    hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, grad=grad,
                       opts=hx.SolverOpts(tol=1e-6, max_cycles=1), raise_on_failure=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, _, infos = hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, grad=grad, opts=opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": "320x320x160 salt model, 27-point, h=15 m, 10 Hz, 8 sources, 300x300 receivers, "
                        "misfit + gradient (8 forward + 8 adjoint ML-GMRES solves to rel.res 1e-6)",
            "solves_per_s": round(2 * nsrc / dt, 4), "s_per_evaluation": round(dt, 3),
            "max_relres_fp64": max(i.relres_fp64 for i in infos),
            "mean_outer_cycles": float(np.mean([i.cycles for i in infos])), "misfit": f}


def sweep(hx, torch, reps, dev):
    """Stencil GB/s over grid sizes (layered-free constant model; the cost of
    the operator does not depend on the model values)."""
    cases = [((64, 64, 64), 16, "7pt"), ((128, 128, 128), 1, "7pt"), ((128, 128, 128), 16, "7pt"),
             ((256, 256, 256), 1, "7pt"), ((256, 256, 256), 8, "7pt"), ((512, 512, 512), 1, "7pt"),
             ((320, 320, 160), 8, "7pt"), ((128, 128, 128), 16, "27pt"), ((320, 320, 160), 8, "27pt")]
    for n, S, sten in cases:
        grid = hx.Grid(n=n, h=15.0, npml=10, v_ref=4500.0, stencil=sten, dtype="c64",
                       w27=(0.5, 0.3, 0.2, 0.6, 0.04, 0.01, 0.005) if sten == "27pt" else (1, 0, 0, 1, 0, 0, 0))
        m_t = torch.full(n, 1.0 / 3000.0 ** 2, dtype=torch.float32, device=dev)
        ms, gbs = apply_timing(hx, torch, grid, m_t, 2 * np.pi * 8.0, S, reps, dev)
        print(json.dumps({"grid": list(n), "rhs": S, "stencil": sten, "us_per_launch": round(ms * 1e3, 1),
                          "GB_s": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}), flush=True)
        torch.cuda.empty_cache()


def extras(hx, torch, workloads, dev):
    """The paths beside the headline step, on the 96^3 FWI workload (h = 30 m,
    layer 10, 5 Hz, 64 sources, 48 x 48 receivers, complex64, ML-GMRES to
    1e-6), each timed warm (its first call builds the solver):
    * the linearised products of pde_derivative over 16 sources (J dm, J^* y,
      H_GN dm, full Hessian dm: 2 / 2 / 3 / 4 solves per source);
    * misfit + gradient with off-grid (windowed-sinc) sources and receivers
      beside the on-node call, all 64 sources;
    * WRI objective + gradient over 16 sources (receiver-space CG capped at 4
      steps: 1 + 2 x 4 solves per source);
    * the inversion driver (fwi_invert): 2 frequencies in one band, 2 draws
      of 16 of the 64 sources, r_sub = 1 (4 L-BFGS iterations per draw);
    * 2.5D misfit + gradient on a 400 x 200 plane (extras_25d)."""
    w = workloads.c3_fwi()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
    opts = hx.SolverOpts(tol=1e-6, max_cycles=30)
    nsrc, nrec = len(w.src), len(w.rec)
    omegas = [2 * np.pi * 4.0, 2 * np.pi * 5.0]
    mt = torch.tensor(w.m_true, dtype=torch.float32, device=dev)
    m_t = torch.tensor(w.m, dtype=torch.float32, device=dev)
    u = torch.empty((2, nsrc) + w.n, dtype=torch.complex64, device=dev)
    hx.misfit_gradient(grid, mt, omegas, w.src, w.rec,
                       torch.zeros((2, nsrc, nrec), dtype=torch.complex64, device=dev),
                       u_store=u, forward_only=True, opts=opts)
    ridx = torch.tensor(w.rec.astype(np.int64), device=dev)
    d2 = u[:, :, ridx[:, 0], ridx[:, 1], ridx[:, 2]].contiguous()
    del u, mt
    torch.cuda.empty_cache()
    d1 = d2[1:2].contiguous()  # 5 Hz
    out = {"workload": "96^3 FWI model (layers + low-velocity sphere), h=30 m, layer 10, complex64, "
                       "ML-GMRES to rel.res 1e-6; data from the true model"}

    def timed(fn):
        fn()  # warm: builds the solver of this problem set
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    rng = np.random.default_rng(workloads.SEED_BASE + 3)
    dm = torch.tensor(workloads.gaussian_random_field(rng, w.n, 4.0) * w.m * 0.02, dtype=torch.float32,
                      device=dev)
    mask16 = np.zeros((1, nsrc), bool)
    mask16[0, ::4] = True
    y = torch.randn((1, nsrc, nrec), dtype=torch.complex64, device=dev) * float(d1.abs().mean())
    progress("extras: pde_derivative products")
    for name, mode, inp, nsol in (("jacobian", "jacobian", dm, 2), ("jacobian_adjoint", "jacobian_adjoint", y, 2),
                                  ("hessian_gn", "hessian_gn", dm, 3), ("hessian", "hessian", dm, 4)):
        dt, _ = timed(lambda: hx.pde_derivative(mode, grid, m_t, w.omega, w.src, w.rec, inp, d=d1, mask=mask16,
                                                opts=opts, raise_on_failure=False))
        out["pde_derivative_" + name] = {"sources": 16, "solves": 16 * nsol, "s": round(dt, 3),
                                         "solves_per_s": round(16 * nsol / dt, 3)}
    progress("extras: off-grid vs on-node misfit + gradient")
    jit = np.random.default_rng(workloads.SEED_BASE + 5)
    src_pos = w.src + np.column_stack([jit.uniform(-0.4, 0.4, (nsrc, 2)), np.zeros(nsrc)])
    rec_pos = w.rec + np.column_stack([jit.uniform(-0.4, 0.4, (nrec, 2)), np.zeros(nrec)])
    sinc = (workloads.SINC_RADIUS, workloads.SINC_KAISER_B)
    dt_on, _ = timed(lambda: hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d1, opts=opts))
    dt_off, _ = timed(lambda: hx.misfit_gradient(grid, m_t, w.omega, src_pos, rec_pos, d1, sinc=sinc, opts=opts))
    out["offgrid_misfit_gradient"] = {"sources": nsrc, "solves": 2 * nsrc, "s": round(dt_off, 3),
                                      "solves_per_s": round(2 * nsrc / dt_off, 3), "on_node_s": round(dt_on, 3),
                                      "sinc": [int(sinc[0]), float(sinc[1])]}
    progress("extras: WRI")
    lam = 3.0 / (12.0 / w.h ** 2 + w.omega ** 2 * float(w.m.max()))  # 3 / (an estimate of ||H||)
    dt, (f, _, infos) = timed(lambda: hx.wri_misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d1, lam,
                                                             mask=mask16, cg_tol=1e-3, cg_max=4, opts=opts,
                                                             raise_on_failure=False))
    sel = [i for k, i in enumerate(infos) if mask16.ravel()[k]]
    nsol = sum(i.matvecs for i in sel)
    out["wri_misfit_gradient"] = {"sources": 16, "lambda": lam, "cg_steps_max": max(i.cycles for i in sel),
                                  "cg_relres_max": max(i.relres_fp64 for i in sel), "solves": int(nsol),
                                  "s": round(dt, 3), "solves_per_s": round(nsol / dt, 3)}
    progress("extras: 2.5D modelling, misfit and gradient")
    out["misfit_gradient_25d"] = extras_25d(hx, torch, workloads, dev, timed)
    progress("extras: inversion driver")
    lo, hi = 1.0 / 4500.0 ** 2, 1.0 / 1500.0 ** 2
    m_run = m_t.clone()

    def run_driver():
        m_run.copy_(m_t)
        return hx.fwi_invert(grid, m_run, omegas, w.src, w.rec, d2, lo, hi, band_size=2, band_overlap=0,
                             r_sub=1, batch=16, subproblems=2, seed=3, opts=opts)
    dt, (draws, recs, _) = timed(run_driver)
    evals = sum(d["evals"] for d in draws)
    out["fwi_invert"] = {"draws": len(draws), "iterations": len(recs), "evaluations": evals,
                         "solves": evals * 2 * 2 * 16, "s": round(dt, 3),
                         "solves_per_s": round(evals * 2 * 2 * 16 / dt, 3),
                         "f_first": draws[0]["f_start"], "f_last": draws[-1]["f_end"]}
    return out


def extras_25d(hx, torch, workloads, dev, timed):
    """2.5D misfit + gradient on a 400 x 200 plane (h = 10 m, layer 20, 8 Hz,
    layered 1500-4000 m/s with 4 % perturbations): 32 sources and 96
    receivers on the plane's top rows at their own offsets along the
    invariant axis, 30 k_y nodes up to 1.5 omega / v_min, so 960 2D problems
    per batched solve (forward and adjoint)."""
    n1, n2, h, npml, f = 400, 200, 10.0, 20, 8.0
    rng = np.random.default_rng(workloads.SEED_BASE + 25)
    depth = np.linspace(0.0, 1.0, n2)
    v = (1500.0 + 2500.0 * depth)[None, None, :] * (1.0 + 0.04 * workloads.gaussian_random_field(rng, (1, n1, n2), 3.0))
    v = np.clip(v, 1500.0, 4500.0)
    grid = hx.Grid(n=(1, n1, n2), h=h, npml=npml, v_ref=float(v.max()), dtype="c64")
    m_t = torch.tensor(1.0 / v ** 2, dtype=torch.float32, device=dev)
    src = np.column_stack([np.linspace(npml + 5, n1 - npml - 6, 32).astype(int), np.full(32, npml + 2)])
    rec = np.column_stack([np.linspace(npml + 2, n1 - npml - 3, 96).astype(int), np.full(96, npml + 1)])
    src_y = np.zeros(32)
    rec_y = np.tile([0.0, 50.0, 100.0], 32)
    om = 2 * np.pi * f
    opts = hx.SolverOpts(tol=1e-6, max_cycles=30)
    kw = dict(nky=30, p_kc=1.5, v_min=1500.0, opts=opts, raise_on_failure=False)
    _, _, d_obs, _ = hx.misfit_gradient_25d(grid, m_t * 1.02, om, src, src_y, rec, rec_y, None, **kw)
    d_obs = d_obs.contiguous()
    dt, (fv, _, _, infos) = timed(lambda: hx.misfit_gradient_25d(grid, m_t, om, src, src_y, rec, rec_y, d_obs, **kw))
    nsol = 2 * 32 * 30
    return {"plane": [n1, n2], "sources": 32, "receivers": 96, "nky": 30, "problems_per_solve": 32 * 30,
            "solves": nsol, "s": round(dt, 3), "solves_per_s": round(nsol / dt, 2),
            "max_relres_fp64": max(i.relres_fp64 for i in infos), "misfit": fv}


def _c4_member(p):
    """One member of the uneven draw as plain arrays (runs in a worker)."""
    import workloads
    w = workloads.c4_problem(p)
    return (tuple(w.n), w.h, w.npml, w.v_ref, w.omega, tuple(int(v) for v in w.src[0]),
            w.m.astype(np.float32))


def _pool_workers():
    """Worker processes for host-side work: the host cores this process may
    use, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def c4_members(params):
    """The members' inputs, built in a pool of fresh (spawned) worker
    processes; the parent has initialised the GPU and does not fork."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(_pool_workers()) as pool:
        return pool.map(_c4_member, params, chunksize=4)


def batched_vs_plain(hx, torch, workloads, count, dev):
    """Solves/s of the uneven batch (the first `count` problems of the seeded
    256-problem draw: dims U{48..160} with aspect <= 2, 3-12 Hz at 8 points
    per wavelength, smooth random 1500-4500 m/s, one source each) solved
    together by helm_solve_batched (in as few batches as fit in device
    memory), and the same problems one at a time by helm_solve.  Both timed
    warm: a one-cycle solve first builds each solver and captures its graph
    (the solver cache ignores the cycle limit), so setup and capture stay
    outside the timed region; same options and tolerance."""
    params = workloads.c4_problem_params(count=256)[:count]
    probs = []
    for n, h, npml, vref, omega, src, m32 in c4_members(params):
        grid = hx.Grid(n=n, h=h, npml=npml, v_ref=vref, dtype="c64")
        m_t = torch.from_numpy(m32).to(dev)
        q_t = torch.zeros(n, dtype=torch.complex64, device=dev)
        q_t[src] = 1.0 / h ** 3
        probs.append((grid, m_t, omega, q_t))
    opts = hx.SolverOpts(tol=1e-6, max_cycles=40)
    warm = hx.SolverOpts(tol=1e-6, max_cycles=1)
    npts = sum(pr[0].N for pr in probs)
    # batches: workspace of the solver + the concatenated right-hand sides,
    # solutions and the caller's u, within 85 % of the free device memory
    free, _ = torch.cuda.mem_get_info(dev)
    budget = 0.85 * free
    batches, cur, used = [], [], 0.0
    for pr in probs:
        need = hx.workspace_bytes(pr[0], opts) + 3 * 8 * pr[0].N
        if cur and used + need > budget:
            batches.append(cur)
            cur, used = [], 0.0
        cur.append(pr)
        used += need
    batches.append(cur)
    tb = 0.0
    binfo = []
    progress(f"uneven batch: {len(probs)} problems ({npts} points) built; {len(batches)} batched solve(s)")
    for b in batches:
        hx.helm_solve_batched(b, opts=warm, raise_on_failure=False)  # setup + capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf = hx.helm_solve_batched(b, opts=opts)
        torch.cuda.synchronize()
        tb += time.perf_counter() - t0
        binfo.extend(inf)
    progress(f"uneven batch: batched {tb:.2f} s; plain solves one at a time")
    tp = 0.0
    pinfo = []
    for ip, pr in enumerate(probs):
        if ip % 32 == 0:
            progress(f"uneven batch: plain problem {ip}/{len(probs)}")
        hx.helm_solve(pr[0], pr[1], pr[2], pr[3], opts=warm, raise_on_failure=False)  # setup + capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf = hx.helm_solve(pr[0], pr[1], pr[2], pr[3], opts=opts)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t0
        pinfo.extend(inf)
    return {
        "workload": f"{'all' if count == 256 else 'first ' + str(count)} of the 256-problem uneven draw "
                    "(dims 48-160, aspect <= 2, 3-12 Hz, 8 ppw at 1500 m/s, layer 8), one source each, "
                    "ML-GMRES to 1e-6",
        "problems": count, "points": int(npts), "batches": len(batches),
        "batched_solves_per_s": round(count / tb, 4), "plain_solves_per_s": round(count / tp, 4),
        "batched_vs_plain": round(tp / tb, 3),
        "batched_s": round(tb, 3), "plain_s": round(tp, 3),
        "max_relres_batched": max(i.relres_fp64 for i in binfo),
        "max_relres_plain": max(i.relres_fp64 for i in pinfo),
        "all_converged": all(i.status == 0 for i in binfo + pinfo),
        "mean_cycles_batched": float(np.mean([i.cycles for i in binfo])),
        "mean_cycles_plain": float(np.mean([i.cycles for i in pinfo])),
    }


def _oracle_step(args):
    """One outer FGMRES step of the oracle (one V-cycle of the preconditioner,
    one operator apply, a modified Gram-Schmidt step) for one source on the
    full grid, BLAS on one thread; returns (seconds, seconds of setup)."""
    n, h, npml, omega, vref, m, src = args
    from threadpoolctl import threadpool_limits
    from oracle import operators as ops
    from oracle import mlgmres, fwi
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        g = ops.make_grid(n, h, npml, omega, vref)
        hier = mlgmres.Hierarchy(g, m, mlgmres.MLOptions())
        q = fwi.point_source(g, tuple(src))
        A = hier.A(0)
        v = q / np.linalg.norm(q)
        t1 = time.perf_counter()
        z = hier.vcycle(0, v)
        wv = A(z)
        wv = wv - np.vdot(v, wv) * v
        _ = wv / np.linalg.norm(wv)
        t2 = time.perf_counter()
    return t2 - t1, t1 - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, m64, src, omega, steps_per_solve):
    """The oracle on the host cores: P worker processes (P = the cores this
    process may use, at most 16), each running one outer FGMRES step of a
    different source on the full grid at the same time (the paper's
    parallelism over sources); throughput = P steps over the wall time of
    the slowest worker's step, converted to solves with the GPU's mean
    number of outer steps per solve."""
    import multiprocessing as mp
    P = _pool_workers()
    jobs = [(tuple(w.n), w.h, w.npml, omega, w.v_ref, m64, tuple(int(v) for v in src[i % len(src)]))
            for i in range(P)]
    progress(f"cpu baseline: {P} oracle workers")
    with mp.get_context("spawn").Pool(P) as pool:
        res = pool.map(_oracle_step, jobs, chunksize=1)
    wall = max(r[0] for r in res)
    return {
        "value": round(P / (wall * steps_per_solve), 6), "unit": "solves/s", "cores": P, "kind": "oracle",
        "cpu": cpu_model(),
        "sample": f"{P} worker processes (BLAS on one thread each), each one outer FGMRES step "
                  f"(one V-cycle + one operator apply + one Gram-Schmidt step) of one source on the full "
                  f"128^3 grid, concurrently; slowest step {wall:.2f} s (mean "
                  f"{np.mean([r[0] for r in res]):.2f} s, setup excluded); scaled by "
                  f"{steps_per_solve:.1f} outer steps per solve (GPU mean)",
    }


def copy_timing(torch, n_elems, reps, dev):
    """Achieved GB/s of a plain device copy of two complex64 buffers of
    n_elems (read + write), HIP events on the current stream: the practical
    ceiling for a streaming kernel."""
    xs = [torch.randn(n_elems, dtype=torch.complex64, device=dev) for _ in range(2)]
    ys = [torch.empty_like(xs[0]) for _ in range(2)]
    for i in range(3):
        ys[i % 2].copy_(xs[i % 2])
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(reps):
        ys[i % 2].copy_(xs[i % 2])
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return ms, 16.0 * n_elems / (ms * 1e-3) / 1e9


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil7_pair_c2_128cube_16rhs_hbm_traffic.txt")
# the kernel (stencil.hip) and its launch / tile choice (operator.hip)
STENCIL_SOURCES = [os.path.join(ROOT, "paper_1703_09268_amd", "csrc", f) for f in ("stencil.hip", "operator.hip")]


def stencil_source_digest():
    import hashlib
    h = hashlib.sha256()
    for path in STENCIL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per stencil launch from the committed hardware-counter
    summary, if it was taken on the current stencil sources (sha256 match);
    otherwise None."""
    try:
        digest = stencil_source_digest()
        with open(TRAFFIC_FILE) as f:
            rec = json.loads([ln for ln in f if ln.startswith("{")][-1])
    except (OSError, ValueError, IndexError):
        return None
    if rec.get("stencil_source_sha256") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def stencil_timing(hx, torch, grid, m_t, w, S, reps, dev):
    """Average duration of the stencil kernel (helm_apply with S right-hand
    sides: one kernel launch each) from HIP events recorded on the launch
    stream; two input/output pairs alternate."""
    xs = [torch.randn((S,) + tuple(w.n), dtype=torch.complex64, device=dev) for _ in range(2)]
    ys = [torch.empty_like(xs[0]) for _ in range(2)]
    for i in range(3):
        hx.helm_apply(grid, m_t, w.omega, xs[i % 2], out=ys[i % 2])
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(reps):
        hx.helm_apply(grid, m_t, w.omega, xs[i % 2], out=ys[i % 2])
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bytes_launch = (16 * S + 4) * w.N
    return ms, bytes_launch / (ms * 1e-3) / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this benchmark measures one GPU only (one process per GPU; the "
              "multi-GPU sharding over (source, frequency) pairs is not part of it). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1703_09268_amd as hx
    import workloads

    dev = torch.device("cuda:0")
    if args.sweep:
        sweep(hx, torch, args.stencil_reps, dev)
        return
    if args.c5_only:
        print(json.dumps(c5_gradient(hx, torch, workloads, dev)), flush=True)
        return
    if args.stencil27_only:
        rec = stencil27_timing(hx, torch, workloads, args.stencil_reps, dev)
        n27 = 8 * 320 * 320 * 160  # the 8 right-hand sides of the 320x320x160 grid
        cms, cgbs = copy_timing(torch, n27, args.stencil_reps, dev)
        rec.update({"copy_ms": cms, "copy_GB_s": cgbs, "copy_bytes_per_launch": 16 * n27})
        print(json.dumps(rec), flush=True)
        return
    if args.batch_only:
        print(json.dumps(batched_vs_plain(hx, torch, workloads, args.batch_count, dev)), flush=True)
        return
    if args.extras_only:
        print(json.dumps(extras(hx, torch, workloads, dev)), flush=True)
        return
    w = workloads.c2_layered()
    if args.stencil_only:
        grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
        m_t = torch.tensor(w.m, dtype=torch.float32, device=dev)
        ms, gbs = stencil_timing(hx, torch, grid, m_t, w, len(w.src), args.stencil_reps, dev)
        cms, cgbs = copy_timing(torch, len(w.src) * w.N, args.stencil_reps, dev)
        print(json.dumps({"stencil_ms_per_launch": ms, "GB_s": gbs, "copy_ms": cms, "copy_GB_s": cgbs,
                          "copy_bytes_per_launch": 16 * len(w.src) * w.N}), flush=True)
        return
    nsrc = len(w.src)
    rec = workloads.surface_positions(w.n, w.npml, (args.nrec, args.nrec))
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
    opts = hx.SolverOpts(tol=1e-6, max_cycles=30)
    m_t = torch.tensor(w.m, dtype=torch.float32, device=dev)
    # observed data: forward-modelled from a perturbed model (untimed input)
    rng = np.random.default_rng(workloads.SEED_BASE + 2)
    m_true = (w.m * (1.0 + 0.02 * workloads.gaussian_random_field(rng, w.n, 4.0)))
    mt_t = torch.tensor(m_true, dtype=torch.float32, device=dev)
    u_true = torch.empty((nsrc,) + w.n, dtype=torch.complex64, device=dev)
    _, _, _ = hx.misfit_gradient(grid, mt_t, w.omega, w.src, rec,
                                 torch.zeros((nsrc, len(rec)), dtype=torch.complex64, device=dev),
                                 u_store=u_true, forward_only=True, opts=opts)
    ridx = torch.tensor(rec.astype(np.int64), device=dev)
    d_t = u_true[:, ridx[:, 0], ridx[:, 1], ridx[:, 2]].contiguous()
    del u_true
    grad = torch.empty(w.n, dtype=torch.float32, device=dev)

    def step():
        return hx.misfit_gradient(grid, m_t, w.omega, w.src, rec, d_t, grad=grad, opts=opts)

    progress("128^3 misfit + gradient: data synthesised; warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    progress(f"128^3 misfit + gradient: {args.steps} timed steps")
    t0 = time.perf_counter()
    infos = []
    fval = None
    for _ in range(args.steps):
        fval, _, inf = step()
        infos.extend(inf)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solves = args.steps * 2 * nsrc
    sps = solves / elapsed
    relres = [i.relres_fp64 for i in infos]
    cycles = [i.cycles for i in infos]

    progress(f"128^3 misfit + gradient: {sps:.3f} solves/s; stencil timings")
    # ---- stencil kernel alone: 16 right-hand sides, HIP events on the stream
    S = nsrc
    st_ms, gbs = stencil_timing(hx, torch, grid, m_t, w, S, args.stencil_reps, dev)
    cp_ms, cp_gbs = copy_timing(torch, S * w.N, args.stencil_reps, dev)
    traffic = measured_traffic()
    st27 = None if args.no_stencil27 else stencil27_timing(hx, torch, workloads, args.stencil_reps, dev)
    if not args.no_c5:
        progress("320x320x160 27-point misfit + gradient")
    c5 = None if args.no_c5 else c5_gradient(hx, torch, workloads, dev)
    if not args.no_batch:
        progress("uneven batch: building problems")
    batch = None if args.no_batch else batched_vs_plain(hx, torch, workloads, args.batch_count, dev)
    if not args.no_extras:
        progress("96^3 derivative products, off-grid geometry, WRI, inversion driver")
    ext = None if args.no_extras else extras(hx, torch, workloads, dev)

    out = {
        "metric": METRIC,
        "value": round(sps, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": "128^3 layered+random, h=12.5 m, 8 Hz, 16 sources, "
                        f"{args.nrec}x{args.nrec} receivers, misfit + gradient "
                        "(16 forward + 16 adjoint ML-GMRES solves to rel.res 1e-6)",
            "grid": list(w.n), "sources": nsrc, "receivers": int(len(rec)),
            "solver": "FGMRES(5) + 3-grid V-cycle (3,5,3,5), complex64, FP64 outer residual",
            "solves_per_step": 2 * nsrc,
        },
        "solve_stats": {
            "max_relres_fp64": max(relres), "mean_outer_cycles": float(np.mean(cycles)),
            "max_outer_cycles": int(max(cycles)), "misfit": fval,
        },
        "batched_vs_plain": batch,
        "stencil": {
            "kernel": "k_h7p<false,false,0,false> (helm_apply: complex64 7-point, pair tiles, 16 rhs)",
            "ms_per_launch": round(st_ms, 5), "GB_s": round(gbs, 1),
            "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_point": f"16*{S}+4",
            "algorithmic_bytes_per_launch": (16 * S + 4) * w.N,
            "copy_ceiling_GB_s": round(cp_gbs, 1),
        },
        "stencil27": st27,
        "c5_27pt_gradient": c5,
        "extras_96cube": ext,
        "roofline": {
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, m_t.double().cpu().numpy(), w.src, w.omega,
                                           5.0 * float(np.mean(cycles)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
