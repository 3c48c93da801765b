"""GPU tests of helm_apply_noalloc, the allocation-free variant of helm_apply
(its operator description lives in the library's fixed per-GPU scratch array):
through the C ABI, two calls in a row (the second with a smaller input, so it
runs on what the first left in the scratch array) against helm_apply on the
same inputs, and against the FP64 oracle; requests beyond the scratch limit
are rejected before any device work."""
import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import operators as ops

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
W27 = workloads.W27_DEFAULT


def _inputs(n, npml, nrhs, dtype, stencil, seed):
    rng = np.random.default_rng(seed)
    v = 1500.0 + 3000.0 * rng.random(n)
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    rdt = torch.float32 if dtype == "c64" else torch.float64
    grid = hx.Grid(n=n, h=20.0, npml=npml, v_ref=float(v.max()), stencil=stencil, dtype=dtype,
                   w27=W27 if stencil == "27pt" else (1, 0, 0, 1, 0, 0, 0))
    m_t = torch.tensor(1.0 / v ** 2, dtype=rdt, device=DEV)
    x_t = torch.tensor(workloads.random_complex(rng, (nrhs,) + tuple(n)), dtype=cdt, device=DEV)
    return grid, m_t, x_t


# (first call: grid, layer, right-hand sides), (second, smaller call)
CASES = [
    ("c64", "7pt", ((40, 36, 34), 5, 3), ((21, 19, 18), 3, 2)),        # pair tiles, interleaved
    ("c64", "7pt", ((128, 128, 128), 15, 16), ((64, 64, 64), 8, 4)),   # the 128^3 x 16 shape
    ("c64", "7pt", ((25, 23, 21), 4, 2), ((13, 12, 11), 2, 1)),        # odd nz: one point per lane
    ("c64", "27pt", ((34, 30, 28), 5, 2), ((20, 18, 16), 3, 1)),       # LDS-staged pair pass
    ("c64", "27pt", ((9, 7, 600), 1, 2), ((8, 6, 400), 1, 1)),         # planes too wide for LDS, then staged
    ("c128", "27pt", ((24, 22, 21), 4, 2), ((15, 14, 13), 2, 1)),      # point-wise map
    ("c128", "7pt", ((30, 26, 22), 4, 2), ((17, 15, 13), 2, 3)),
]


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("dtype,stencil,first,second", CASES,
                         ids=[f"{c[0]}-{c[1]}-{'x'.join(map(str, c[2][0]))}" for c in CASES])
def test_noalloc_matches_helm_apply_two_calls(dtype, stencil, first, second, adjoint):
    tol = 1e-5 if dtype == "c64" else 1e-12
    for k, (n, npml, nrhs) in enumerate((first, second)):
        print(f"case noalloc {dtype} {stencil} adj={adjoint} call {k} n={n} nrhs={nrhs}", flush=True)
        grid, m_t, x_t = _inputs(n, npml, nrhs, dtype, stencil, seed=sum(n) + 7 * k)
        y_ref = hx.helm_apply(grid, m_t, 2 * np.pi * 6.0, x_t, adjoint=adjoint)
        y_na = torch.full_like(x_t, float("nan"))
        hx.helm_apply_noalloc(grid, m_t, 2 * np.pi * 6.0, x_t, y_na, adjoint=adjoint)
        torch.cuda.synchronize()
        a = y_na.cpu().numpy().astype(np.complex128)
        b = y_ref.cpu().numpy().astype(np.complex128)
        assert np.all(np.isfinite(a))
        diff = np.abs(a - b).max()
        print(f"  max |noalloc - helm_apply| = {diff:.3e} (bitwise equal: {bool(diff == 0)})", flush=True)
        assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b)
        # and against the oracle on one right-hand side
        g = ops.make_grid(n, grid.h, npml, 2 * np.pi * 6.0, grid.v_ref)
        ref = ops.apply(g, m_t.cpu().numpy().astype(np.float64), x_t[-1].cpu().numpy().astype(np.complex128),
                        adjoint=adjoint, stencil=stencil, w27=grid.w27)
        assert np.linalg.norm(a[-1] - ref) <= tol * np.linalg.norm(ref)


def test_noalloc_rejects_requests_beyond_the_scratch_array():
    """40000 right-hand sides of a complex128 27-point 16^3 operator need
    about 11 MB of descriptors and maps (limit 8 MiB): HELM_E_INVAL, and the
    output is untouched."""
    grid, m_t, _ = _inputs((16, 16, 16), 2, 1, "c128", "27pt", seed=3)
    nrhs = 40000
    x_t = torch.zeros((nrhs, 16, 16, 16), dtype=torch.complex128, device=DEV)
    y_t = torch.full_like(x_t, 7.0)
    print("case noalloc rejection", flush=True)
    with pytest.raises(hx.HelmError) as e:
        hx.helm_apply_noalloc(grid, m_t, 2 * np.pi * 6.0, x_t, y_t)
    assert e.value.status == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y_t == 7.0).all())
