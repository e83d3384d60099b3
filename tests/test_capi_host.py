"""Host-only checks of the C ABI: the library loads, exports every function
include/llg.h declares, and rejects invalid arguments before touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "llg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "sizeof")))


@pytest.fixture(scope="module")
def lib():
    from paper_2607_15290_amd import _lib
    return _lib.load()


def test_header_lists_the_five_path_entry_points():
    names = declared_functions()
    for n in ("llg_matvec", "fft_hss_apply", "gmres_solve", "llg_step_euler", "llg_step_midpoint"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_signatures_cover_header():
    from paper_2607_15290_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_ctx_create_rejects_bad_sizes(lib):
    h = ctypes.c_void_p()
    # odd nx, factors other than 2, 3, 5, a 7 or 9 factor, sizes out of range, bad h
    for nx, ny, nz, hh in [(3, 4, 1, 0.1), (4, 14, 1, 0.1), (1024, 4, 1, 0.1), (4, 4, 2, 0.1), (4, 4, 1, 0.0),
                           (4, 4, 1, -1.0), (8, 8, 3, 0.1), (0, 8, 1, 0.1), (18, 8, 1, 0.1), (8, 8, 36, 0.1),
                           (768, 8, 1, 0.1), (8, 640, 1, 0.1), (24, 2, 1, 0.1), (8, 8, 1, float("nan"))]:
        assert lib.llg_ctx_create(ctypes.byref(h), nx, ny, nz, hh, 0) == 1, (nx, ny, nz, hh)
        assert h.value is None
        assert len(lib.llg_last_error()) > 0
    assert lib.llg_ctx_create(None, 8, 8, 1, 0.1, 0) == 1
    for lens in [(0.0, 1.0, 1.0), (1.0, -1.0, 1.0), (1.0, 1.0, 0.0), (1.0, float("inf"), 1.0)]:
        assert lib.llg_ctx_create_cell(ctypes.byref(h), 8, 8, 1, *lens, 0) == 1
        assert h.value is None


def test_entry_points_reject_null_context(lib):
    from paper_2607_15290_amd import _lib
    p = _lib.LLGParams()
    p.alpha, p.cexc, p.dt, p.theta, p.shift = 0.1, 1.0, 1e-3, 1.0, 0.5
    assert lib.llg_matvec(None, ctypes.byref(p), None, None, None, 0, None) == 1
    assert lib.fft_hss_apply(None, ctypes.byref(p), None, None, None, 0, None) == 1
    o = _lib.LLGSolverOpts()
    o.restart, o.maxiter, o.rtol = 30, 100, 1e-10
    assert lib.gmres_solve(None, ctypes.byref(p), None, None, None, ctypes.byref(o), None, None, 0, None) == 1
    assert lib.llg_step_euler(None, ctypes.byref(p), None, None, None, ctypes.byref(o), None, None, 0, None) == 1
    assert lib.llg_step_midpoint(None, ctypes.byref(p), None, None, None, 1e-10, 10, ctypes.byref(o), None, None,
                                 0, None) == 1
    assert lib.llg_workspace_bytes(None, 30, 0) == 0
    assert lib.llg_ctx_destroy(None) == 0
    assert lib.llg_precond_op(None, ctypes.byref(p), None, None, None, None, 0, 0, None, None) == 1
    assert lib.llg_precond_op_f32(None, ctypes.byref(p), None, None, None, None, 0, None, 0, 0, None, None) == 1
    assert lib.gmres_solve_noalloc(None, ctypes.byref(p), None, None, None, ctypes.byref(o), None, None) == 1


def test_binding_refuses_unaligned_tensors():
    """The binding passes only 16-byte aligned device addresses to the C ABI
    (the library also refuses others with LLG_EARG)."""
    import torch
    from paper_2607_15290_amd.llg import aligned_ptr
    t = torch.zeros(64, dtype=torch.float64)
    assert aligned_ptr(t) == t.data_ptr()
    with pytest.raises(ValueError):
        aligned_ptr(t[1:])


def test_binding_structs_match_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct (compiled with gcc here)."""
    import shutil
    import subprocess
    from paper_2607_15290_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"llg_params": _lib.LLGParams, "llg_solver_opts": _lib.LLGSolverOpts,
               "llg_solver_stats": _lib.LLGSolverStats, "llg_step_stats": _lib.LLGStepStats,
               "llg_kernel_profile": _lib.LLGKernelProfile}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "llg.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
