"""Write tests/golden/precond_cycles.json: outer FGMRES(5) cycle counts and
per-cycle relative residuals of the oracle's ML-GMRES solve (ML-GMRES
section: FGMRES with 5 inner iterations to relative residual 1e-6, V-cycle
with (3, 5, 3, 5) GMRES smoothers / coarse solves, 3 grids) on seeded
workloads, for the GPU test that compares the library's cycle counts with
them.  Calls only the oracle and the seeded input generators; inputs are
rounded to what a complex64 solve receives (model to float32, right-hand
side to complex64).  Run from the repository root:
    python tests/golden/make_precond_cycles.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import fwi, mlgmres  # noqa: E402
from oracle import operators as ops  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precond_cycles.json")


def case_inputs(c):
    """Seeded workload of a case (shared with the GPU test)."""
    if c["kind"] == "constant":
        nl, ppw, v0, f = c["n_lambda"], c["ppw"], 2000.0, 5.0
        n = nl * ppw + 1 + 2 * ppw
        w = workloads.constant_workload((n, n, n), v0 / (f * ppw), ppw, f, v0=v0, dtype="c64")
    else:
        w = workloads.layered_random_workload(tuple(c["n"]), c["h"], c["npml"], c["freq"],
                                              nsrc_xy=(1, 1), seed=c["seed"])
    if c["stencil"] == "27pt":
        w.stencil = "27pt"
        w.w27 = workloads.W27_DEFAULT
    return w


CASES = [
    {"name": "constant 57^3 (n_lambda 5, 8 ppw), 7-point", "kind": "constant", "n_lambda": 5, "ppw": 8,
     "stencil": "7pt", "adjoint": False},
    {"name": "layered 48x44x40, 7-point", "kind": "layered", "n": [48, 44, 40], "h": 20.0, "npml": 6,
     "freq": 6.0, "seed": 61, "stencil": "7pt", "adjoint": False},
    {"name": "layered 48x44x40, 7-point, adjoint", "kind": "layered", "n": [48, 44, 40], "h": 20.0, "npml": 6,
     "freq": 6.0, "seed": 61, "stencil": "7pt", "adjoint": True},
    {"name": "layered 40x36x38, 27-point", "kind": "layered", "n": [40, 36, 38], "h": 20.0, "npml": 5,
     "freq": 6.0, "seed": 62, "stencil": "27pt", "adjoint": False},
    {"name": "layered 40x36x38, 27-point, adjoint", "kind": "layered", "n": [40, 36, 38], "h": 20.0, "npml": 5,
     "freq": 6.0, "seed": 62, "stencil": "27pt", "adjoint": True},
]


def main():
    rows = []
    for c in CASES:
        w = case_inputs(c)
        g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
        m = w.m.astype(np.float32).astype(np.float64)
        q = fwi.point_source(g, tuple(w.src[0])).astype(np.complex64).astype(np.complex128)
        hist = []
        _, info = mlgmres.mlgmres_solve(g, m, q, tol=1e-6, max_cycles=30, stencil=w.stencil, w27=w.w27,
                                        adjoint=c["adjoint"], history=hist)
        row = dict(c)
        row.update({"grid": list(w.n), "oracle_cycles": info["cycles"], "oracle_relres": hist})
        print(row["name"], info, flush=True)
        rows.append(row)
    with open(OUT, "w") as fh:
        json.dump({"written_by": "tests/golden/make_precond_cycles.py (oracle only)",
                   "solver": "FGMRES(5) + 3-grid V-cycle (3,5,3,5), tol 1e-6, x0 = 0",
                   "cases": rows}, fh, indent=1)


if __name__ == "__main__":
    main()
