"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/helm.h declares, and the host-only entry points behave (no GPU
compute is launched here)."""
import ctypes as C
import os
import re

import pytest

from paper_1703_09268_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:helm_status|size_t|void|const char\*)\s+(\w+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libhelm.so is not built (run __graft_entry__.build())")
    return L.load()


def test_header_declarations_match_export_list():
    assert _declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_version_and_default_options(lib):
    assert lib.helm_version().decode().startswith("helm-gfx950")
    o = L.helm_solver_opts()
    lib.helm_default_opts(C.byref(o))
    assert (o.method, o.restart, o.ks_o, o.ks_i, o.kc_o, o.kc_i, o.levels) == \
        (L.HELM_FGMRES_ML, 5, 3, 5, 3, 5, 3)
    assert o.tol == 1e-6


def _grid(n=(32, 32, 32), npml=8, dtype=L.HELM_C64):
    g = L.helm_grid()
    for a in range(3):
        g.n[a] = n[a]
    g.h, g.npml, g.pml_R, g.v_ref = 10.0, npml, 1e-3, 2000.0
    g.stencil, g.dtype = L.HELM_7PT, dtype
    return g


def test_workspace_bytes_and_invalid_grids(lib):
    o = L.helm_solver_opts()
    lib.helm_default_opts(C.byref(o))
    g = _grid()
    b1 = lib.helm_workspace_bytes(C.byref(g), C.byref(o), 1)
    b4 = lib.helm_workspace_bytes(C.byref(g), C.byref(o), 4)
    N = 32 ** 3
    # within the paper's 26-vector bound plus the FP64 outer iterate
    assert 18 * N * 8 < b1 <= (26 + 2) * N * 8
    assert 3.9 * b1 < b4 < 4.1 * b1
    bad = _grid(npml=16)  # npml >= n/2
    assert lib.helm_workspace_bytes(C.byref(bad), C.byref(o), 1) == 0
    small = _grid(n=(2, 32, 32), npml=0)
    assert lib.helm_workspace_bytes(C.byref(small), C.byref(o), 1) == 0
    assert lib.helm_workspace_bytes(C.byref(g), C.byref(o), 0) == 0


def test_null_context_is_rejected(lib):
    g = _grid()
    st = lib.helm_apply(None, C.byref(g), None, 1.0, 0, 1, None, None, None)
    assert st == L.HELM_E_INVAL
    assert b"context" in lib.helm_last_error(None)
