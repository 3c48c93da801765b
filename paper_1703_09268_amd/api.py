"""Python binding of the C ABI (argument marshalling only).

Every function checks tensor placement, dtype, shape and contiguity, then
calls the entry point of the same name in ``libhelm.so`` on the current
torch stream.  All arithmetic happens in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


class HelmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


@dataclass
class Grid:
    """Mirror of ``helm_grid``: grid incl. absorbing layer, z fastest."""

    n: Sequence[int]
    h: float
    npml: int
    v_ref: float
    pml_R: float = 1e-3
    stencil: str = "7pt"  # "7pt" | "27pt"
    dtype: str = "c64"  # "c64" | "c128"
    w27: Sequence[float] = (1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0)

    @property
    def N(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def complex_dtype(self):
        return torch.complex64 if self.dtype == "c64" else torch.complex128

    @property
    def real_dtype(self):
        return torch.float32 if self.dtype == "c64" else torch.float64

    def c_struct(self) -> L.helm_grid:
        g = L.helm_grid()
        for a in range(3):
            g.n[a] = int(self.n[a])
        g.h = float(self.h)
        g.npml = int(self.npml)
        g.pml_R = float(self.pml_R)
        g.v_ref = float(self.v_ref)
        g.stencil = {"7pt": L.HELM_7PT, "27pt": L.HELM_27PT}[self.stencil]
        g.dtype = {"c64": L.HELM_C64, "c128": L.HELM_C128}[self.dtype]
        for c in range(7):
            g.w27[c] = float(self.w27[c])
        return g


@dataclass
class SolverOpts:
    """Mirror of ``helm_solver_opts``; defaults are the paper's settings."""

    method: str = "fgmres_ml"  # "fgmres_ml" | "gmres"
    restart: int = 5
    max_cycles: int = 50
    tol: float = 1e-6
    ks_o: int = 3
    ks_i: int = 5
    kc_o: int = 3
    kc_i: int = 5
    levels: int = 3
    warm_start: bool = False

    def c_struct(self) -> L.helm_solver_opts:
        o = L.helm_solver_opts()
        o.method = {"gmres": L.HELM_GMRES, "fgmres_ml": L.HELM_FGMRES_ML}[self.method]
        o.restart, o.max_cycles, o.tol = int(self.restart), int(self.max_cycles), float(self.tol)
        o.ks_o, o.ks_i, o.kc_o, o.kc_i = int(self.ks_o), int(self.ks_i), int(self.kc_o), int(self.kc_i)
        o.levels = int(self.levels)
        o.warm_start = int(bool(self.warm_start))
        return o


@dataclass
class SolveInfo:
    status: int
    cycles: int
    inner_its: int
    matvecs: int
    relres_fp64: float

    @property
    def status_name(self):
        return L.STATUS_NAMES.get(self.status, str(self.status))


_ctx = {}


def _context(device: int) -> C.c_void_p:
    lib = L.load()
    if device not in _ctx:
        h = C.c_void_p()
        st = lib.helm_create(C.byref(h), int(device))
        if st != L.HELM_OK:
            raise HelmError(st, lib.helm_last_error(None).decode())
        _ctx[device] = h
    return _ctx[device]


def _check(ctx, st, allow=(L.HELM_OK,)):
    if st not in allow:
        raise HelmError(st, L.load().helm_last_error(ctx).decode())
    return st


def _dev_tensor(t: torch.Tensor, dtype, numel, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a torch tensor on a GPU")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _nrhs(x: torch.Tensor, N: int) -> int:
    if x.numel() % N != 0 or x.numel() == 0:
        raise ValueError(f"array of {x.numel()} elements is not a whole number of grids of {N}")
    return x.numel() // N


def helm_apply(grid: Grid, m: torch.Tensor, omega: float, x: torch.Tensor,
               adjoint: bool = False, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = H(m) x or H(m)^H x for x of shape (..., nx, ny, nz)."""
    dev = x.device.index or 0
    nrhs = _nrhs(x, grid.N)
    if out is None:
        out = torch.empty_like(x)
    ctx = _context(dev)
    g = grid.c_struct()
    st = L.load().helm_apply(
        ctx, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), float(omega),
        int(bool(adjoint)), nrhs, _dev_tensor(x, grid.complex_dtype, nrhs * grid.N, "x"),
        _dev_tensor(out, grid.complex_dtype, nrhs * grid.N, "out"), _stream(dev))
    _check(ctx, st)
    return out


def helm_apply_noalloc(grid: Grid, m: torch.Tensor, omega: float, x: torch.Tensor,
                       out: torch.Tensor, adjoint: bool = False) -> torch.Tensor:
    """helm_apply through the allocation-free entry point: ``out`` must be
    given (the call allocates nothing, here or in the library)."""
    dev = x.device.index or 0
    nrhs = _nrhs(x, grid.N)
    ctx = _context(dev)
    g = grid.c_struct()
    st = L.load().helm_apply_noalloc(
        ctx, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), float(omega),
        int(bool(adjoint)), nrhs, _dev_tensor(x, grid.complex_dtype, nrhs * grid.N, "x"),
        _dev_tensor(out, grid.complex_dtype, nrhs * grid.N, "out"), _stream(dev))
    _check(ctx, st)
    return out


def helm_solve(grid: Grid, m: torch.Tensor, omega: float, q: torch.Tensor,
               adjoint: bool = False, opts: Optional[SolverOpts] = None,
               u: Optional[torch.Tensor] = None, raise_on_failure: bool = True):
    """Solve H u = q (or H^H u = q) for q of shape (..., nx, ny, nz).

    Returns (u, [SolveInfo per right-hand side])."""
    dev = q.device.index or 0
    nrhs = _nrhs(q, grid.N)
    opts = opts or SolverOpts()
    if u is None:
        if opts.warm_start:
            raise ValueError("warm_start needs u")
        u = torch.empty_like(q)
    infos = (L.helm_solve_info * nrhs)()
    ctx = _context(dev)
    g, o = grid.c_struct(), opts.c_struct()
    st = L.load().helm_solve(
        ctx, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), float(omega),
        int(bool(adjoint)), nrhs, _dev_tensor(q, grid.complex_dtype, nrhs * grid.N, "q"),
        _dev_tensor(u, grid.complex_dtype, nrhs * grid.N, "u"), C.byref(o), infos, _stream(dev))
    allow = (L.HELM_OK,) if raise_on_failure else (L.HELM_OK, L.HELM_NOT_CONVERGED, L.HELM_BREAKDOWN)
    _check(ctx, st, allow)
    return u, [SolveInfo(i.status, i.cycles, i.inner_its, i.matvecs, i.relres_fp64) for i in infos]


def helm_solve_batched(problems, adjoint: bool = False, opts: Optional[SolverOpts] = None,
                       raise_on_failure: bool = True):
    """Solve a batch of independent problems of different sizes together.

    problems: sequence of (grid, m, omega, q[, u]) with torch device tensors
    (all grids of one dtype and stencil).  Returns ([u], [SolveInfo])."""
    if not problems:
        raise ValueError("empty batch")
    opts = opts or SolverOpts()
    arr = (L.helm_problem * len(problems))()
    outs = []
    dev = problems[0][1].device.index or 0
    for i, pr in enumerate(problems):
        grid, m, omega, q = pr[0], pr[1], pr[2], pr[3]
        u = pr[4] if len(pr) > 4 and pr[4] is not None else None
        if u is None:
            if opts.warm_start:
                raise ValueError("warm_start needs u for every problem")
            u = torch.empty_like(q)
        arr[i].grid = grid.c_struct()
        arr[i].m = _dev_tensor(m, grid.real_dtype, grid.N, "m")
        arr[i].omega = float(omega)
        arr[i].q = _dev_tensor(q, grid.complex_dtype, grid.N, "q")
        arr[i].u = _dev_tensor(u, grid.complex_dtype, grid.N, "u")
        outs.append(u)
    infos = (L.helm_solve_info * len(problems))()
    ctx = _context(dev)
    o = opts.c_struct()
    st = L.load().helm_solve_batched(ctx, len(problems), arr, int(bool(adjoint)), C.byref(o), infos,
                                     _stream(dev))
    allow = (L.HELM_OK,) if raise_on_failure else (L.HELM_OK, L.HELM_NOT_CONVERGED, L.HELM_BREAKDOWN)
    _check(ctx, st, allow)
    return outs, [SolveInfo(i.status, i.cycles, i.inner_its, i.matvecs, i.relres_fp64) for i in infos]


def _idx_array(pos):
    return np.ascontiguousarray(np.asarray(pos, dtype=np.int32).reshape(-1, 3))


def _points(src, rec, sinc):
    """Host arrays of the source and receiver geometry: on-node int32 indices
    (sinc None), or float64 positions in node units for the windowed-sinc
    entry points (sinc = (radius, kaiser_b))."""
    if sinc is None:
        for name, a in (("src", src), ("rec", rec)):
            if not np.issubdtype(np.asarray(a).dtype, np.integer):
                raise ValueError(f"{name}: off-grid positions need sinc=(radius, kaiser_b)")
        return _idx_array(src), _idx_array(rec), C.POINTER(C.c_int32)
    conv = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3))
    return conv(src), conv(rec), C.POINTER(C.c_double)


def misfit_gradient(grid: Grid, m: torch.Tensor, omega, src, rec, d: torch.Tensor,
                    src_amp=None, mask=None, grad: Optional[torch.Tensor] = None, sinc=None,
                    u_store: Optional[torch.Tensor] = None, forward_only: bool = False,
                    reuse_u: bool = False, accumulate: bool = False, u_fp64: bool = False,
                    renormalise: bool = False, opts: Optional[SolverOpts] = None,
                    raise_on_failure: bool = True):
    """Misfit f = 1/2 sum ||P_r u - d||^2 over the selected (frequency,
    source) pairs and its gradient w.r.t. m.

    omega: one angular frequency or a sequence of nfreq; src, rec: (nsrc, 3)
    / (nrec, 3) integer node indices (host); d: complex device tensor of
    nfreq * nsrc * nrec values ([frequency][source][receiver]); src_amp:
    complex amplitudes broadcastable to (nfreq, nsrc); mask: booleans
    (nfreq, nsrc) selecting the pairs (default all).  u_store (optional,
    [nfreq][nsrc][N]) receives or, with reuse_u, supplies the forward fields;
    with u_fp64 it is complex128 (the FP64 outer iterates).  renormalise
    divides f and g by the number of selected pairs.  Returns (f, grad,
    infos): infos per pair, forward solves then adjoint solves (only those
    that ran), [frequency][source] order, zero entries for unselected pairs.
    sinc=(radius, kaiser_b): src / rec are positions in node units anywhere
    inside the grid, interpolated by Kaiser-windowed sincs
    (misfit_gradient_offgrid)."""
    if (u_fp64 or reuse_u) and u_store is None:
        raise ValueError("u_fp64 and reuse_u need u_store")
    dev = m.device.index or 0
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, dtype=np.float64)).ravel())
    nfreq = len(om)
    src_a, rec_a, PT = _points(src, rec, sinc)
    nsrc, nrec = len(src_a), len(rec_a)
    amp_p = None
    if src_amp is not None:
        amp = np.broadcast_to(np.asarray(src_amp, np.complex128), (nfreq, nsrc))
        amp_d = np.ascontiguousarray(np.stack([amp.real, amp.imag], axis=-1).ravel())
        amp_p = amp_d.ctypes.data_as(C.POINTER(C.c_double))
    mask_p = None
    if mask is not None:
        mask_a = np.ascontiguousarray(
            np.broadcast_to(np.asarray(mask, bool), (nfreq, nsrc)).astype(np.uint8))
        mask_p = mask_a.ctypes.data_as(C.POINTER(C.c_uint8))
    flags = (L.HELM_MG_FORWARD_ONLY if forward_only else 0) | \
        (L.HELM_MG_REUSE_U if reuse_u else 0) | (L.HELM_MG_ACCUMULATE if accumulate else 0) | \
        (L.HELM_MG_U_FP64 if u_fp64 else 0) | (L.HELM_MG_RENORMALISE if renormalise else 0)
    u_dtype = torch.complex128 if u_fp64 else grid.complex_dtype
    if grad is None and not forward_only:
        grad = torch.empty(tuple(grid.n), dtype=grid.real_dtype, device=m.device)
    opts = opts or SolverOpts()
    npair = nfreq * nsrc
    infos = (L.helm_solve_info * (2 * npair))()
    f = C.c_double(0.0)
    ctx = _context(dev)
    g, o = grid.c_struct(), opts.c_struct()
    geo = (nrec, rec_a.ctypes.data_as(PT)) if sinc is None else \
        (nrec, rec_a.ctypes.data_as(PT), int(sinc[0]), float(sinc[1]))
    fn = L.load().misfit_gradient if sinc is None else L.load().misfit_gradient_offgrid
    st = fn(
        ctx, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), nfreq,
        om.ctypes.data_as(C.POINTER(C.c_double)), nsrc,
        src_a.ctypes.data_as(PT), amp_p, mask_p, *geo,
        _dev_tensor(d, grid.complex_dtype, npair * nrec, "d"), C.byref(f),
        None if grad is None else _dev_tensor(grad, grid.real_dtype, grid.N, "grad"),
        None if u_store is None else _dev_tensor(u_store, u_dtype, npair * grid.N, "u_store"),
        flags, C.byref(o), infos, _stream(dev))
    allow = (L.HELM_OK,) if raise_on_failure else (L.HELM_OK, L.HELM_NOT_CONVERGED, L.HELM_BREAKDOWN)
    _check(ctx, st, allow)
    nsolve = npair if (forward_only or reuse_u) else 2 * npair
    first = npair if reuse_u else 0
    inf = [SolveInfo(i.status, i.cycles, i.inner_its, i.matvecs, i.relres_fp64)
           for i in list(infos)[first:first + nsolve]]
    return f.value, grad, inf


_MODES = {"jacobian": L.HELM_JACOB_FORW, "jacobian_adjoint": L.HELM_JACOB_ADJ,
          "hessian_gn": L.HELM_HESS_GN, "hessian": L.HELM_HESS}


def pde_derivative(mode: str, grid: Grid, m: torch.Tensor, omega, src, rec, input: torch.Tensor,
                   d: Optional[torch.Tensor] = None, src_amp=None, mask=None,
                   out: Optional[torch.Tensor] = None, u_store: Optional[torch.Tensor] = None,
                   reuse_u: bool = False, u_fp64: bool = False, accumulate: bool = False,
                   renormalise: bool = False, opts: Optional[SolverOpts] = None,
                   raise_on_failure: bool = True, sinc=None):
    """Linearised products over the selected (frequency, source) pairs.

    mode: "jacobian" (J dm -> [nfreq][nsrc][nrec] complex), "jacobian_adjoint"
    (J^* y, y [nfreq][nsrc][nrec] -> model), "hessian_gn" (J^* J dm) or
    "hessian" (full Hessian of the misfit with observed data d, applied to
    dm).  Other arguments as in misfit_gradient.  Returns (out, infos): infos
    per solve (forward fields first, then the mode's solves), each
    [frequency][source] (zero entries for unselected pairs / solves not run)."""
    if mode not in _MODES:
        raise ValueError(f"mode must be one of {sorted(_MODES)}")
    md = _MODES[mode]
    if (u_fp64 or reuse_u) and u_store is None:
        raise ValueError("u_fp64 and reuse_u need u_store")
    if md == L.HELM_HESS and d is None:
        raise ValueError("the full Hessian needs the observed data d")
    dev = m.device.index or 0
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, dtype=np.float64)).ravel())
    nfreq = len(om)
    src_a, rec_a, PT = _points(src, rec, sinc)
    nsrc, nrec = len(src_a), len(rec_a)
    npair = nfreq * nsrc
    amp_p = None
    if src_amp is not None:
        amp = np.broadcast_to(np.asarray(src_amp, np.complex128), (nfreq, nsrc))
        amp_d = np.ascontiguousarray(np.stack([amp.real, amp.imag], axis=-1).ravel())
        amp_p = amp_d.ctypes.data_as(C.POINTER(C.c_double))
    mask_p = None
    if mask is not None:
        mask_a = np.ascontiguousarray(
            np.broadcast_to(np.asarray(mask, bool), (nfreq, nsrc)).astype(np.uint8))
        mask_p = mask_a.ctypes.data_as(C.POINTER(C.c_uint8))
    flags = (L.HELM_MG_REUSE_U if reuse_u else 0) | (L.HELM_MG_ACCUMULATE if accumulate else 0) | \
        (L.HELM_MG_U_FP64 if u_fp64 else 0) | (L.HELM_MG_RENORMALISE if renormalise else 0)
    if md == L.HELM_JACOB_ADJ:
        in_p = _dev_tensor(input, grid.complex_dtype, npair * nrec, "input")
    else:
        in_p = _dev_tensor(input, grid.real_dtype, grid.N, "input")
    if out is None:
        out = (torch.empty((nfreq, nsrc, nrec), dtype=grid.complex_dtype, device=m.device)
               if md == L.HELM_JACOB_FORW else
               torch.empty(tuple(grid.n), dtype=grid.real_dtype, device=m.device))
    out_p = (_dev_tensor(out, grid.complex_dtype, npair * nrec, "out") if md == L.HELM_JACOB_FORW
             else _dev_tensor(out, grid.real_dtype, grid.N, "out"))
    u_dtype = torch.complex128 if u_fp64 else grid.complex_dtype
    opts = opts or SolverOpts()
    infos = (L.helm_solve_info * (4 * npair))()
    ctx = _context(dev)
    g, o = grid.c_struct(), opts.c_struct()
    geo = (nrec, rec_a.ctypes.data_as(PT)) if sinc is None else \
        (nrec, rec_a.ctypes.data_as(PT), int(sinc[0]), float(sinc[1]))
    fn = L.load().pde_derivative if sinc is None else L.load().pde_derivative_offgrid
    st = fn(
        ctx, md, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), nfreq,
        om.ctypes.data_as(C.POINTER(C.c_double)), nsrc,
        src_a.ctypes.data_as(PT), amp_p, mask_p, *geo, in_p,
        None if d is None else _dev_tensor(d, grid.complex_dtype, npair * nrec, "d"), out_p,
        None if u_store is None else _dev_tensor(u_store, u_dtype, npair * grid.N, "u_store"),
        flags, C.byref(o), infos, _stream(dev))
    allow = (L.HELM_OK,) if raise_on_failure else (L.HELM_OK, L.HELM_NOT_CONVERGED, L.HELM_BREAKDOWN)
    _check(ctx, st, allow)
    nsolve = {L.HELM_JACOB_FORW: 2, L.HELM_JACOB_ADJ: 2, L.HELM_HESS_GN: 3, L.HELM_HESS: 4}[md]
    inf = [[SolveInfo(i.status, i.cycles, i.inner_its, i.matvecs, i.relres_fp64)
            for i in list(infos)[k * npair:(k + 1) * npair]] for k in range(nsolve)]
    return out, inf


def wri_misfit_gradient(grid: Grid, m: torch.Tensor, omega, src, rec, d: torch.Tensor, lam: float,
                        src_amp=None, mask=None, grad: Optional[torch.Tensor] = None,
                        u_store: Optional[torch.Tensor] = None, forward_only: bool = False,
                        accumulate: bool = False, u_fp64: bool = False, renormalise: bool = False,
                        cg_tol: float = 1e-6, cg_max: int = 200, opts: Optional[SolverOpts] = None,
                        raise_on_failure: bool = True):
    """WRI (penalty method) objective and gradient over the selected
    (frequency, source) pairs (wri_misfit_gradient): the arguments of
    misfit_gradient (on-node geometry) plus the penalty weight lam and the
    receiver-space CG's tolerance and step limit.  Returns (f, grad, infos)
    with one SolveInfo per pair ([frequency][source] order) describing its
    CG: status, cycles = CG steps, matvecs = ML-GMRES solves, relres = the
    CG's final relative residual."""
    if u_fp64 and u_store is None:
        raise ValueError("u_fp64 needs u_store")
    dev = m.device.index or 0
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, dtype=np.float64)).ravel())
    nfreq = len(om)
    src_a, rec_a, PT = _points(src, rec, None)
    nsrc, nrec = len(src_a), len(rec_a)
    amp_p = None
    if src_amp is not None:
        amp = np.broadcast_to(np.asarray(src_amp, np.complex128), (nfreq, nsrc))
        amp_d = np.ascontiguousarray(np.stack([amp.real, amp.imag], axis=-1).ravel())
        amp_p = amp_d.ctypes.data_as(C.POINTER(C.c_double))
    mask_p = None
    if mask is not None:
        mask_a = np.ascontiguousarray(np.broadcast_to(np.asarray(mask, bool), (nfreq, nsrc)).astype(np.uint8))
        mask_p = mask_a.ctypes.data_as(C.POINTER(C.c_uint8))
    flags = (L.HELM_MG_FORWARD_ONLY if forward_only else 0) | (L.HELM_MG_ACCUMULATE if accumulate else 0) | \
        (L.HELM_MG_U_FP64 if u_fp64 else 0) | (L.HELM_MG_RENORMALISE if renormalise else 0)
    if grad is None and not forward_only:
        grad = torch.empty(tuple(grid.n), dtype=grid.real_dtype, device=m.device)
    opts = opts or SolverOpts()
    npair = nfreq * nsrc
    infos = (L.helm_solve_info * npair)()
    f = C.c_double(0.0)
    ctx = _context(dev)
    g, o = grid.c_struct(), opts.c_struct()
    u_dtype = torch.complex128 if u_fp64 else grid.complex_dtype
    st = L.load().wri_misfit_gradient(
        ctx, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), nfreq,
        om.ctypes.data_as(C.POINTER(C.c_double)), nsrc, src_a.ctypes.data_as(PT), amp_p, mask_p, nrec,
        rec_a.ctypes.data_as(PT), _dev_tensor(d, grid.complex_dtype, npair * nrec, "d"), float(lam),
        float(cg_tol), int(cg_max), C.byref(f),
        None if grad is None else _dev_tensor(grad, grid.real_dtype, grid.N, "grad"),
        None if u_store is None else _dev_tensor(u_store, u_dtype, npair * grid.N, "u_store"),
        flags, C.byref(o), infos, _stream(dev))
    allow = (L.HELM_OK,) if raise_on_failure else (L.HELM_OK, L.HELM_NOT_CONVERGED, L.HELM_BREAKDOWN)
    _check(ctx, st, allow)
    inf = [SolveInfo(i.status, i.cycles, i.inner_its, i.matvecs, i.relres_fp64) for i in infos]
    return f.value, grad, inf


def misfit_gradient_25d(grid: Grid, m: torch.Tensor, omega, src, src_y, rec, rec_y,
                        d: Optional[torch.Tensor] = None, nky: int = 40, p_kc: float = 1.0,
                        v_min: float = 1500.0, src_amp=None, mask=None, grad: Optional[torch.Tensor] = None,
                        want_data: bool = True, forward_only: bool = False, accumulate: bool = False,
                        renormalise: bool = False, opts: Optional[SolverOpts] = None,
                        raise_on_failure: bool = True):
    """2.5D modelling, misfit and gradient (misfit_gradient_25d) on a 2D grid
    (grid.n[0] == 1).  src, rec: (n, 2) plane nodes; src_y, rec_y: their
    coordinates along the invariant axis (m); d: observed data
    [nfreq][nsrc][nrec] (None: modelling only).  Returns (f, grad, d_pred,
    infos): d_pred [nfreq][nsrc][nrec] (None unless want_data), infos per
    2D solve, forward then adjoint, [frequency][source][k_y] order."""
    dev = m.device.index or 0
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, dtype=np.float64)).ravel())
    nfreq = len(om)
    src_a = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1, 2))
    rec_a = np.ascontiguousarray(np.asarray(rec, dtype=np.int32).reshape(-1, 2))
    nsrc, nrec = len(src_a), len(rec_a)
    sy = np.ascontiguousarray(np.asarray(src_y, dtype=np.float64).reshape(nsrc))
    ry = np.ascontiguousarray(np.asarray(rec_y, dtype=np.float64).reshape(nrec))
    amp_p = None
    if src_amp is not None:
        amp = np.broadcast_to(np.asarray(src_amp, np.complex128), (nfreq, nsrc))
        amp_d = np.ascontiguousarray(np.stack([amp.real, amp.imag], axis=-1).ravel())
        amp_p = amp_d.ctypes.data_as(C.POINTER(C.c_double))
    mask_p = None
    if mask is not None:
        mask_a = np.ascontiguousarray(np.broadcast_to(np.asarray(mask, bool), (nfreq, nsrc)).astype(np.uint8))
        mask_p = mask_a.ctypes.data_as(C.POINTER(C.c_uint8))
    if d is None:
        forward_only = True
    flags = (L.HELM_MG_FORWARD_ONLY if forward_only else 0) | (L.HELM_MG_ACCUMULATE if accumulate else 0) | \
        (L.HELM_MG_RENORMALISE if renormalise else 0)
    if grad is None and not forward_only:
        grad = torch.empty(tuple(grid.n), dtype=grid.real_dtype, device=m.device)
    d_pred = torch.zeros((nfreq, nsrc, nrec), dtype=grid.complex_dtype, device=m.device) if want_data else None
    opts = opts or SolverOpts()
    infos = (L.helm_solve_info * (2 * nfreq * nsrc * int(nky)))()
    f = C.c_double(0.0)
    ctx = _context(dev)
    g, o = grid.c_struct(), opts.c_struct()
    PI = C.POINTER(C.c_int32)
    PD = C.POINTER(C.c_double)
    st = L.load().misfit_gradient_25d(
        ctx, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), nfreq, om.ctypes.data_as(PD), int(nky),
        float(p_kc), float(v_min), nsrc, src_a.ctypes.data_as(PI), sy.ctypes.data_as(PD), amp_p, mask_p, nrec,
        rec_a.ctypes.data_as(PI), ry.ctypes.data_as(PD),
        None if d is None else _dev_tensor(d, grid.complex_dtype, nfreq * nsrc * nrec, "d"), C.byref(f),
        None if grad is None else _dev_tensor(grad, grid.real_dtype, grid.N, "grad"),
        None if d_pred is None else _dev_tensor(d_pred, grid.complex_dtype, nfreq * nsrc * nrec, "d_pred"),
        flags, C.byref(o), infos, _stream(dev))
    allow = (L.HELM_OK,) if raise_on_failure else (L.HELM_OK, L.HELM_NOT_CONVERGED, L.HELM_BREAKDOWN)
    _check(ctx, st, allow)
    inf = [SolveInfo(i.status, i.cycles, i.inner_its, i.matvecs, i.relres_fp64) for i in infos]
    return f.value, grad, d_pred, inf


def fwi_invert(grid: Grid, m: torch.Tensor, omega, src, rec, d: torch.Tensor, lo, hi,
               src_amp=None, band_size: int = 4, band_overlap: int = 2, r_sub: int = 20,
               memory: int = 5, batch: int = 0, subproblems: int = 1, batch_increase: int = 1,
               seed: int = 0, c1: float = 1e-4, max_ls: int = 10, gtol: float = 1e-6,
               step0: Optional[float] = None, sinc=None, opts: Optional[SolverOpts] = None,
               max_records: int = 100000, raise_on_failure: bool = False):
    """Inversion by frequency continuation, stochastic source subsets and a
    box-constrained L-BFGS (fwi_invert / fwi_invert_offgrid); m (device,
    the grid's real dtype) is overwritten by the result.

    lo, hi: floats, or float64 device tensors of N values (lo = hi clamps a
    point).  step0 defaults to 5 % of the range the bounds span,
    max(hi) - min(lo).  The other
    arguments are those of misfit_gradient and of ``helm_fwi_params``.
    Returns (draws, records, sources): one dict per draw, one dict per
    L-BFGS iteration (the first max_records), and the sources of every draw
    ([draws][nsrc], -1 padded)."""
    dev = m.device.index or 0
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, dtype=np.float64)).ravel())
    nfreq = len(om)
    src_a, rec_a, PT = _points(src, rec, sinc)
    nsrc, nrec = len(src_a), len(rec_a)
    amp_p = None
    if src_amp is not None:
        amp = np.broadcast_to(np.asarray(src_amp, np.complex128), (nfreq, nsrc))
        amp_d = np.ascontiguousarray(np.stack([amp.real, amp.imag], axis=-1).ravel())
        amp_p = amp_d.ctypes.data_as(C.POINTER(C.c_double))
    bounds = []
    for b in (lo, hi):
        if isinstance(b, torch.Tensor):
            bounds.append((_dev_tensor(b, torch.float64, grid.N, "bound"), 0.0))
        else:
            bounds.append((None, float(b)))
    if step0 is None:
        width = [float((b.max() if i else -b.min()).item()) if isinstance(b, torch.Tensor) else
                 (float(b) if i else -float(b)) for i, b in enumerate((lo, hi))]
        step0 = 0.05 * (width[0] + width[1])
    p = L.helm_fwi_params(band_size, band_overlap, r_sub, memory, batch, subproblems, batch_increase,
                          max_ls, seed & ((1 << 64) - 1), c1, gtol, float(step0), bounds[0][1], bounds[1][1])
    lib = L.load()
    ndraw = lib.helm_fwi_draw_count(nfreq, C.byref(p))
    if ndraw < 0:
        raise HelmError(L.HELM_E_INVAL, "invalid inversion parameters")
    draws = (L.helm_fwi_draw * ndraw)()
    sources = np.full(ndraw * nsrc, -1, np.int32)
    recs = (L.helm_fwi_record * max(1, max_records))()
    nrecs = C.c_int(0)
    opts = opts or SolverOpts()
    ctx = _context(dev)
    g, o = grid.c_struct(), opts.c_struct()
    geo = (nrec, rec_a.ctypes.data_as(PT)) if sinc is None else \
        (nrec, rec_a.ctypes.data_as(PT), int(sinc[0]), float(sinc[1]))
    fn = lib.fwi_invert if sinc is None else lib.fwi_invert_offgrid
    st = fn(ctx, C.byref(g), _dev_tensor(m, grid.real_dtype, grid.N, "m"), bounds[0][0], bounds[1][0], nfreq,
            om.ctypes.data_as(C.POINTER(C.c_double)), nsrc, src_a.ctypes.data_as(PT), amp_p, *geo,
            _dev_tensor(d, grid.complex_dtype, nfreq * nsrc * nrec, "d"), C.byref(p), C.byref(o), draws,
            sources.ctypes.data_as(C.POINTER(C.c_int32)), recs, max_records, C.byref(nrecs), _stream(dev))
    allow = (L.HELM_OK,) if raise_on_failure else (L.HELM_OK, L.HELM_NOT_CONVERGED, L.HELM_BREAKDOWN)
    _check(ctx, st, allow)
    fields = lambda s: {k: getattr(s, k) for k, _ in s._fields_ if k != "pad_"}
    return ([fields(x) for x in draws], [fields(x) for x in list(recs)[:min(nrecs.value, max_records)]],
            sources.reshape(ndraw, nsrc))


def version() -> str:
    return L.load().helm_version().decode()


def workspace_bytes(grid: Grid, opts: Optional[SolverOpts] = None, nrhs: int = 1) -> int:
    g, o = grid.c_struct(), (opts or SolverOpts()).c_struct()
    return int(L.load().helm_workspace_bytes(C.byref(g), C.byref(o), int(nrhs)))
