"""ctypes declarations of the C ABI in ``include/helm.h``.

Loading fails loudly (RuntimeError) when ``libhelm.so`` has not been built:
there is no fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelm.so")

HELM_OK = 0
HELM_NOT_CONVERGED = 1
HELM_BREAKDOWN = 2
HELM_E_INVAL = -1
HELM_E_NOMEM = -2
HELM_E_HIP = -3
HELM_E_UNSUPPORTED = -4

HELM_C64, HELM_C128 = 0, 1
HELM_7PT, HELM_27PT = 0, 1
HELM_GMRES, HELM_FGMRES_ML = 0, 1

HELM_MG_FORWARD_ONLY = 1
HELM_MG_REUSE_U = 2
HELM_MG_ACCUMULATE = 4
HELM_MG_U_FP64 = 8
HELM_MG_RENORMALISE = 16

HELM_JACOB_FORW = 1
HELM_JACOB_ADJ = 2
HELM_HESS_GN = 3
HELM_HESS = 4

STATUS_NAMES = {
    HELM_OK: "HELM_OK",
    HELM_NOT_CONVERGED: "HELM_NOT_CONVERGED",
    HELM_BREAKDOWN: "HELM_BREAKDOWN",
    HELM_E_INVAL: "HELM_E_INVAL",
    HELM_E_NOMEM: "HELM_E_NOMEM",
    HELM_E_HIP: "HELM_E_HIP",
    HELM_E_UNSUPPORTED: "HELM_E_UNSUPPORTED",
}

# every entry point declared in include/helm.h
EXPORTS = ("helm_create", "helm_destroy", "helm_last_error", "helm_version",
           "helm_default_opts", "helm_workspace_bytes", "helm_apply",
           "helm_apply_noalloc", "helm_solve", "helm_solve_batched", "misfit_gradient",
           "misfit_gradient_offgrid", "pde_derivative", "pde_derivative_offgrid",
           "helm_fwi_draw_count", "fwi_invert", "fwi_invert_offgrid", "wri_misfit_gradient",
           "misfit_gradient_25d")


class helm_grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("npml", C.c_int32),
                ("pml_R", C.c_double), ("v_ref", C.c_double),
                ("stencil", C.c_int32), ("dtype", C.c_int32),
                ("w27", C.c_double * 7)]


class helm_solver_opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("restart", C.c_int32),
                ("max_cycles", C.c_int32), ("tol", C.c_double),
                ("ks_o", C.c_int32), ("ks_i", C.c_int32), ("kc_o", C.c_int32),
                ("kc_i", C.c_int32), ("levels", C.c_int32),
                ("warm_start", C.c_int32)]


class helm_problem(C.Structure):
    _fields_ = [("grid", helm_grid), ("m", C.c_void_p), ("omega", C.c_double),
                ("q", C.c_void_p), ("u", C.c_void_p)]


class helm_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32),
                ("inner_its", C.c_int32), ("pad_", C.c_int32),
                ("matvecs", C.c_int64), ("relres_fp64", C.c_double)]


class helm_fwi_params(C.Structure):
    _fields_ = [("band_size", C.c_int32), ("band_overlap", C.c_int32), ("r_sub", C.c_int32),
                ("memory", C.c_int32), ("batch", C.c_int32), ("subproblems", C.c_int32),
                ("batch_increase", C.c_int32), ("max_ls", C.c_int32), ("seed", C.c_uint64),
                ("c1", C.c_double), ("gtol", C.c_double), ("step0", C.c_double),
                ("lo", C.c_double), ("hi", C.c_double)]


class helm_fwi_draw(C.Structure):
    _fields_ = [("band", C.c_int32), ("draw", C.c_int32), ("nsel", C.c_int32),
                ("max_iters", C.c_int32), ("iters", C.c_int32), ("failed", C.c_int32),
                ("evals", C.c_int32), ("status", C.c_int32), ("f_start", C.c_double),
                ("f_end", C.c_double)]


class helm_fwi_record(C.Structure):
    _fields_ = [("band", C.c_int32), ("draw", C.c_int32), ("iter", C.c_int32), ("nsel", C.c_int32),
                ("trials", C.c_int32), ("accepted", C.c_int32), ("status", C.c_int32),
                ("pad_", C.c_int32), ("f", C.c_double), ("f_new", C.c_double), ("step", C.c_double),
                ("pgmax", C.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libhelm.so (once) and declare the prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    vp, i32, dbl = C.c_void_p, C.c_int, C.c_double
    G, O, I = C.POINTER(helm_grid), C.POINTER(helm_solver_opts), C.POINTER(helm_solve_info)
    lib.helm_create.argtypes = [C.POINTER(vp), i32]
    lib.helm_destroy.argtypes = [vp]
    lib.helm_last_error.argtypes = [vp]
    lib.helm_last_error.restype = C.c_char_p
    lib.helm_version.restype = C.c_char_p
    lib.helm_default_opts.argtypes = [O]
    lib.helm_default_opts.restype = None
    lib.helm_workspace_bytes.argtypes = [G, O, i32]
    lib.helm_workspace_bytes.restype = C.c_size_t
    lib.helm_apply.argtypes = [vp, G, vp, dbl, i32, i32, vp, vp, vp]
    lib.helm_apply_noalloc.argtypes = [vp, G, vp, dbl, i32, i32, vp, vp, vp]
    lib.helm_solve.argtypes = [vp, G, vp, dbl, i32, i32, vp, vp, O, I, vp]
    lib.helm_solve_batched.argtypes = [vp, i32, C.POINTER(helm_problem), i32, O, I, vp]
    lib.misfit_gradient.argtypes = [vp, G, vp, i32, C.POINTER(C.c_double), i32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                    C.POINTER(C.c_uint8), i32, C.POINTER(C.c_int32), vp,
                                    C.POINTER(C.c_double), vp, vp, i32, O, I, vp]
    lib.pde_derivative.argtypes = [vp, i32, G, vp, i32, C.POINTER(C.c_double), i32,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                   C.POINTER(C.c_uint8), i32, C.POINTER(C.c_int32), vp, vp,
                                   vp, vp, i32, O, I, vp]
    D = C.POINTER(C.c_double)
    lib.misfit_gradient_offgrid.argtypes = [vp, G, vp, i32, D, i32, D, D, C.POINTER(C.c_uint8), i32, D,
                                            i32, dbl, vp, D, vp, vp, i32, O, I, vp]
    lib.pde_derivative_offgrid.argtypes = [vp, i32, G, vp, i32, D, i32, D, D, C.POINTER(C.c_uint8), i32, D,
                                           i32, dbl, vp, vp, vp, vp, i32, O, I, vp]
    lib.wri_misfit_gradient.argtypes = [vp, G, vp, i32, D, i32, C.POINTER(C.c_int32), D,
                                        C.POINTER(C.c_uint8), i32, C.POINTER(C.c_int32), vp, dbl, dbl, i32,
                                        D, vp, vp, i32, O, I, vp]
    lib.misfit_gradient_25d.argtypes = [vp, G, vp, i32, D, i32, dbl, dbl, i32, C.POINTER(C.c_int32), D, D,
                                        C.POINTER(C.c_uint8), i32, C.POINTER(C.c_int32), D, vp, D, vp, vp, i32,
                                        O, I, vp]
    P = C.POINTER(helm_fwi_params)
    lib.helm_fwi_draw_count.argtypes = [i32, P]
    lib.helm_fwi_draw_count.restype = C.c_int
    FW = [C.POINTER(helm_fwi_draw), C.POINTER(C.c_int32), C.POINTER(helm_fwi_record), i32,
          C.POINTER(C.c_int), vp]
    lib.fwi_invert.argtypes = [vp, G, vp, vp, vp, i32, D, i32, C.POINTER(C.c_int32), D, i32,
                               C.POINTER(C.c_int32), vp, P, O] + FW
    lib.fwi_invert_offgrid.argtypes = [vp, G, vp, vp, vp, i32, D, i32, D, D, i32, D, i32, dbl, vp, P,
                                       O] + FW
    for name in ("helm_create", "helm_destroy", "helm_apply", "helm_apply_noalloc", "helm_solve",
                 "helm_solve_batched", "misfit_gradient", "misfit_gradient_offgrid", "pde_derivative",
                 "pde_derivative_offgrid", "fwi_invert", "fwi_invert_offgrid", "wri_misfit_gradient",
           "misfit_gradient_25d"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
