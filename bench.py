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
    p.add_argument("--batch-count", type=int, default=64,
                   help="problems of the uneven 256-problem draw used for batched vs plain")
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--stencil-only", action="store_true",
                   help="only the stencil measurement (for hardware-counter runs)")
    p.add_argument("--sweep", action="store_true",
                   help="only the stencil size sweep (7-point 64^3..512^3, 27-point), one JSON line per size")
    p.add_argument("--no-stencil27", action="store_true")
    p.add_argument("--c5", action="store_true",
                   help="also time the 320x320x160 27-point misfit + gradient (about 75 s more)")
    p.add_argument("--c5-only", action="store_true")
    p.add_argument("--stencil27-only", action="store_true",
                   help="only the 27-point operator timing on the 320x320x160 workload (and a plain "
                        "copy of the same size, the calibration of hardware-counter runs)")
    p.add_argument("--batch-only", action="store_true", help="only batched vs plain")
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
    hx.misfit_gradient(grid, m_t, w.omega, w.src, w.rec, d_t, grad=grad, opts=opts)  # build + warm
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


def batched_vs_plain(hx, torch, workloads, count, dev):
    """Solves/s of the uneven batch (first `count` problems of the seeded
    256-problem draw: dims U{48..160} with aspect <= 2, 3-12 Hz at 8 points
    per wavelength, smooth random 1500-4500 m/s, one source each) solved
    together by helm_solve_batched, and the same problems one at a time by
    helm_solve.  Both timed warm (second call, setup and graph capture
    outside the timed region), same options and tolerance."""
    params = workloads.c4_problem_params(count=256)[:count]
    probs = []
    for p in params:
        w = workloads.c4_problem(p)
        grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
        m_t = torch.tensor(w.m, dtype=torch.float32, device=dev)
        q_t = torch.zeros(w.n, dtype=torch.complex64, device=dev)
        i, j, k = (int(v) for v in w.src[0])
        q_t[i, j, k] = 1.0 / w.h ** 3
        probs.append((grid, m_t, w.omega, q_t))
    opts = hx.SolverOpts(tol=1e-6, max_cycles=40)
    npts = sum(pr[0].N for pr in probs)
    hx.helm_solve_batched(probs, opts=opts)  # setup + capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, binfo = hx.helm_solve_batched(probs, opts=opts)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    tp = 0.0
    pinfo = []
    for pr in probs:
        hx.helm_solve(pr[0], pr[1], pr[2], pr[3], opts=opts)  # setup + capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf = hx.helm_solve(pr[0], pr[1], pr[2], pr[3], opts=opts)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t0
        pinfo.extend(inf)
    return {
        "workload": f"first {count} of the 256-problem uneven draw (dims 48-160, aspect <= 2, "
                    "3-12 Hz, 8 ppw at 1500 m/s, layer 8), one source each, ML-GMRES to 1e-6",
        "problems": count, "points": int(npts),
        "batched_solves_per_s": round(count / tb, 4), "plain_solves_per_s": round(count / tp, 4),
        "batched_vs_plain": round(tp / tb, 3),
        "batched_s": round(tb, 3), "plain_s": round(tp, 3),
        "max_relres_batched": max(i.relres_fp64 for i in binfo),
        "max_relres_plain": max(i.relres_fp64 for i in pinfo),
        "all_converged": all(i.status == 0 for i in binfo + pinfo),
        "mean_cycles_batched": float(np.mean([i.cycles for i in binfo])),
    }


def cpu_baseline(w, m32, src, rec, omega, target_s=0.0):
    """Oracle timing on a bounded sample: outer FGMRES Arnoldi steps (one
    V-cycle + one operator apply + modified Gram-Schmidt each) of one source
    on the full grid, extrapolated to one solve with the GPU's mean outer
    step count."""
    from oracle import operators as ops
    from oracle import mlgmres, fwi
    g = ops.make_grid(w.n, w.h, w.npml, omega, w.v_ref)
    hier = mlgmres.Hierarchy(g, m32, mlgmres.MLOptions())
    q = fwi.point_source(g, tuple(src[0]))
    A = hier.A(0)
    t0 = time.perf_counter()
    steps = 0
    v = q / np.linalg.norm(q)
    basis = [v]
    while True:
        z = hier.vcycle(0, v)
        wv = A(z)
        for b in basis:
            wv = wv - np.vdot(b, wv) * b
        v = wv / np.linalg.norm(wv)
        basis.append(v)
        steps += 1
        if time.perf_counter() - t0 >= target_s or steps >= 1:
            break
    dt = (time.perf_counter() - t0) / steps
    return dt, steps


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
        print("bench.py: this build measures one GPU only (one process per GPU; the "
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
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

    # ---- stencil kernel alone: 16 right-hand sides, HIP events on the stream
    S = nsrc
    st_ms, gbs = stencil_timing(hx, torch, grid, m_t, w, S, args.stencil_reps, dev)
    cp_ms, cp_gbs = copy_timing(torch, S * w.N, args.stencil_reps, dev)
    traffic = measured_traffic()
    st27 = None if args.no_stencil27 else stencil27_timing(hx, torch, workloads, args.stencil_reps, dev)
    c5 = c5_gradient(hx, torch, workloads, dev) if args.c5 else None
    batch = None if args.no_batch else batched_vs_plain(hx, torch, workloads, args.batch_count, dev)

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
        "roofline": {
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
        },
    }
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):  # the oracle as written, one core
            dt, nst = cpu_baseline(w, m_t.double().cpu().numpy(), w.src, rec, w.omega)
        steps_per_solve = 5.0 * float(np.mean(cycles))
        out["cpu_baseline"] = {
            "value": round(1.0 / (dt * steps_per_solve), 6), "unit": "solves/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{nst} outer FGMRES steps (V-cycle + apply + MGS) of one source on the "
                      f"full 128^3 grid, {dt:.2f} s/step, scaled by {steps_per_solve:.1f} steps "
                      "per solve (GPU mean)",
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
