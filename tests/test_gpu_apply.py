"""GPU parity of helm_apply (7-point and 27-point, forward and adjoint,
complex64 and complex128) against the FP64 oracle, element by element, on
grids that span several tiles with ragged tails; adjoint identity on the GPU."""
import numpy as np
import pytest
import torch

import paper_1703_09268_amd as hx
import workloads
from oracle import operators as ops

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
W27 = workloads.W27_DEFAULT


def _case(n, npml, seed, f=6.0, h=20.0):
    rng = np.random.default_rng(seed)
    v = 1500.0 + 3000.0 * rng.random(n)
    m = 1.0 / v ** 2
    return rng, m, float(v.max()), 2 * np.pi * f, h


def _to_dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("n,npml,nrhs", [((70, 37, 67), 6, 2), ((9, 13, 20), 2, 3),
                                         ((33, 17, 129), 5, 1), ((21, 35, 46), 4, 2),
                                         ((7, 11, 4), 0, 2), ((6, 5, 600), 1, 2)])
def test_apply_matches_oracle(dtype, stencil, adjoint, n, npml, nrhs):
    print(f"case apply dtype={dtype} stencil={stencil} adj={adjoint} n={n}", flush=True)
    rng, m, vref, omega, h = _case(n, npml, seed=sum(n) + nrhs)
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    rdt = torch.float32 if dtype == "c64" else torch.float64
    grid = hx.Grid(n=n, h=h, npml=npml, v_ref=vref, stencil=stencil, dtype=dtype,
                   w27=W27 if stencil == "27pt" else (1, 0, 0, 1, 0, 0, 0))
    x = workloads.random_complex(rng, (nrhs,) + n)
    m_t = _to_dev(m, rdt)
    x_t = _to_dev(x, cdt)
    y_t = hx.helm_apply(grid, m_t, omega, x_t, adjoint=adjoint)
    torch.cuda.synchronize()
    y = y_t.cpu().numpy().astype(np.complex128)
    # the oracle sees exactly the values the GPU saw
    m_used = m_t.cpu().numpy().astype(np.float64)
    x_used = x_t.cpu().numpy().astype(np.complex128)
    g = ops.make_grid(n, h, npml, omega, vref)
    tol = 1e-5 if dtype == "c64" else 1e-12
    for r in range(nrhs):
        ref = ops.apply(g, m_used, x_used[r], adjoint=adjoint, stencil=stencil, w27=grid.w27)
        err = np.abs(y[r] - ref)
        assert np.linalg.norm(err) <= tol * np.linalg.norm(ref)
        assert err.max() <= 4 * tol * np.abs(ref).max()


@pytest.mark.parametrize("adjoint", [False, True])
def test_apply_unaligned_buffers(adjoint):
    """Buffers that start 8 bytes off a 16-byte boundary (a view into a larger
    tensor) take the one-point-per-lane kernel; results match the aligned call
    and the oracle."""
    n, npml, nrhs = (12, 18, 24), 3, 2
    rng, m, vref, omega, h = _case(n, npml, seed=77)
    grid = hx.Grid(n=n, h=h, npml=npml, v_ref=vref, dtype="c64")
    x = workloads.random_complex(rng, (nrhs,) + n)
    m_t = _to_dev(m, torch.float32)
    x_t = _to_dev(x, torch.complex64)
    big = torch.zeros(x_t.numel() + 1, dtype=torch.complex64, device=DEV)
    big[1:] = x_t.flatten()
    x_off = big[1:].view(x_t.shape)
    assert x_off.data_ptr() % 16 == 8
    y_a = hx.helm_apply(grid, m_t, omega, x_t, adjoint=adjoint)
    y_u = hx.helm_apply(grid, m_t, omega, x_off, adjoint=adjoint)
    torch.cuda.synchronize()
    d = torch.linalg.norm(y_a - y_u).item() / torch.linalg.norm(y_a).item()
    assert d <= 1e-6
    g = ops.make_grid(n, h, npml, omega, vref)
    ref = ops.apply(g, m_t.cpu().numpy().astype(np.float64), x_t.cpu().numpy().astype(np.complex128)[1],
                    adjoint=adjoint)
    assert np.linalg.norm(y_u.cpu().numpy()[1] - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_adjoint_identity_on_gpu_fp64(stencil):
    """<H x, y> = <x, H^H y> with both products computed by the library in
    complex128 (paper's adjoint test)."""
    n, npml = (40, 36, 44), 6
    rng, m, vref, omega, h = _case(n, npml, seed=5)
    grid = hx.Grid(n=n, h=h, npml=npml, v_ref=vref, stencil=stencil, dtype="c128",
                   w27=W27 if stencil == "27pt" else (1, 0, 0, 1, 0, 0, 0))
    m_t = _to_dev(m, torch.float64)
    x_t = _to_dev(workloads.random_complex(rng, n), torch.complex128)
    y_t = _to_dev(workloads.random_complex(rng, n), torch.complex128)
    hx_t = hx.helm_apply(grid, m_t, omega, x_t)
    hy_t = hx.helm_apply(grid, m_t, omega, y_t, adjoint=True)
    a = torch.vdot(y_t.flatten(), hx_t.flatten()).item()
    b = torch.vdot(hy_t.flatten(), x_t.flatten()).item()
    den = torch.linalg.norm(hx_t).item() * torch.linalg.norm(y_t).item()
    assert abs(a - b) / den <= 1e-12


def test_apply_full_size_sampled_rows():
    """At the 128^3 layered workload size (16 right-hand sides, the launch
    configuration the solver uses), sampled output rows equal the oracle's
    row-by-row evaluation."""
    w = workloads.c2_layered()
    grid = hx.Grid(n=w.n, h=w.h, npml=w.npml, v_ref=w.v_ref, dtype="c64")
    rng = np.random.default_rng(3)
    nrhs = 16
    m_t = _to_dev(w.m, torch.float32)
    x_t = (torch.randn((nrhs,) + w.n, dtype=torch.complex64, device=DEV))
    y_t = hx.helm_apply(grid, m_t, w.omega, x_t)
    torch.cuda.synchronize()
    g = ops.make_grid(w.n, w.h, w.npml, w.omega, w.v_ref)
    m_used = m_t.cpu().numpy().astype(np.float64)
    for r in (0, 7, 15):
        x_r = x_t[r].cpu().numpy().astype(np.complex128)
        ref = ops.apply7(g, m_used, x_r)
        y_r = y_t[r].cpu().numpy().astype(np.complex128)
        idx = tuple(rng.integers(0, w.n[a], 4096) for a in range(3))
        err = np.abs(y_r[idx] - ref[idx])
        assert err.max() <= 4e-5 * np.abs(ref).max()
        assert np.linalg.norm(y_r - ref) <= 1e-5 * np.linalg.norm(ref)


def test_apply_rejects_bad_arguments():
    n = (16, 16, 16)
    grid = hx.Grid(n=n, h=10.0, npml=8, v_ref=2000.0)  # npml >= n/2
    m_t = torch.ones(n, dtype=torch.float32, device=DEV)
    x_t = torch.zeros(n, dtype=torch.complex64, device=DEV)
    with pytest.raises(hx.HelmError) as e:
        hx.helm_apply(grid, m_t, 1.0, x_t)
    assert e.value.status == -1
    grid = hx.Grid(n=n, h=10.0, npml=2, v_ref=2000.0)
    with pytest.raises(hx.HelmError):
        hx.helm_apply(grid, m_t, -1.0, x_t)


def test_tile_choice_recorded_on_disk(tmp_path, monkeypatch):
    """The tile tuner writes its choice (x chunk, segment order) to the cache
    file named by HELM_TUNE_CACHE, keyed by the device and the segment
    shapes; the operator's values do not depend on the tiles (no reductions),
    so the tuned launch equals a launch with fixed heuristic tiles bit for bit."""
    path = tmp_path / "tiles.tsv"
    n = (41, 29, 34)  # a shape no other test uses
    rng, m, vref, omega, h = _case(n, 4, seed=77)
    grid = hx.Grid(n=n, h=h, npml=4, v_ref=vref, dtype="c64")
    m_t = _to_dev(m, torch.float32)
    x_t = _to_dev(workloads.random_complex(rng, (3,) + n), torch.complex64)
    monkeypatch.setenv("HELM_TUNE_CACHE", str(path))
    y1 = hx.helm_apply(grid, m_t, omega, x_t)
    torch.cuda.synchronize()
    lines = [ln.split("\t") for ln in path.read_text().splitlines()]
    mine = [ln for ln in lines if "41x29x34" in ln[0]]
    assert len(mine) == 1 and mine[0][0].startswith("tiles3|gfx") and "|apply|" in mine[0][0]
    assert int(mine[0][1]) >= 4 and mine[0][2] in ("1", "2", "3")  # segments per tile group
    monkeypatch.setenv("HELM_AUTOTUNE", "0")
    # another operator in between, so that the next call rebuilds this one
    # (now with the heuristic tiles) instead of reusing the tuned one
    y2 = hx.helm_apply(grid, m_t, omega * (1 + 1e-15), x_t)
    y3 = hx.helm_apply(grid, m_t, omega, x_t)
    torch.cuda.synchronize()
    assert torch.equal(y1, y3)
    assert y2.shape == y1.shape


@pytest.mark.parametrize("stencil", ["7pt", "27pt"])
def test_tile_groups_give_the_same_values(stencil, monkeypatch):
    """Five right-hand sides sharing grid and model, their tiles taken
    segment-major, in groups of 2 (the last group ragged), of 3 and all
    interleaved: only the workgroup order changes, so the operator's values
    are bitwise those of the segment-major order."""
    n = (23, 19, 36)
    rng, m, vref, omega, h = _case(n, 3, seed=91)
    grid = hx.Grid(n=n, h=h, npml=3, v_ref=vref, dtype="c64", stencil=stencil)
    m_t = _to_dev(m, torch.float32)
    x_t = _to_dev(workloads.random_complex(rng, (5,) + n), torch.complex64)
    monkeypatch.setenv("HELM_AUTOTUNE", "0")
    ys = []
    for group in ("1", "2", "3", "5"):
        print(f"case tile group {group} {stencil}", flush=True)
        monkeypatch.setenv("HELM_TILE_GROUP", group)
        hx.helm_apply(grid, m_t, omega * (1 + 1e-15), x_t)  # evicts the cached operator
        ys.append(hx.helm_apply(grid, m_t, omega, x_t))
    torch.cuda.synchronize()
    for y in ys[1:]:
        assert torch.equal(y, ys[0])
