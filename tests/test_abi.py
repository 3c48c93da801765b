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
    names = re.findall(r"\b(?:helm_status|size_t|void|int|const char\*)\s+(\w+)\s*\(", text)
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


def _fwi_params(**kw):
    p = L.helm_fwi_params(4, 2, 20, 5, 0, 1, 1, 10, 0, 1e-4, 1e-6, 1e-8, 0.0, 1.0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_fwi_draw_count(lib):
    """bands x draws: 10 frequencies in bands of 4 overlapping by 2 give 4
    bands (the 2D example's layout); 11 give 5; invalid parameters -1."""
    cnt = lambda nf, **kw: lib.helm_fwi_draw_count(nf, C.byref(_fwi_params(**kw)))
    assert cnt(10) == 4 and cnt(11) == 5 and cnt(3) == 1
    assert cnt(10, subproblems=3) == 12
    assert cnt(5, band_size=1, band_overlap=0) == 5
    assert cnt(10, band_overlap=4) == -1 and cnt(10, memory=17) == -1 and cnt(0) == -1
    assert cnt(10, step0=0.0) == -1 and cnt(10, c1=1.0) == -1


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof / offsetof of every struct of include/helm.h, compiled by the
    host C compiler, equal the ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"helm_grid": L.helm_grid, "helm_solver_opts": L.helm_solver_opts,
               "helm_solve_info": L.helm_solve_info, "helm_problem": L.helm_problem,
               "helm_fwi_params": L.helm_fwi_params, "helm_fwi_draw": L.helm_fwi_draw,
               "helm_fwi_record": L.helm_fwi_record}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "helm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"
