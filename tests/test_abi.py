"""The C-ABI library loads and exports every symbol include/peifem.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "peifem.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pe_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("pe_init_grid", "pe_phi_tables", "pe_fine_propagate", "pe_coarse_sweep",
                     "pe_parareal_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2412_01138_amd import peifem
    lib = peifem.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(peifem.EXPORTS) <= set(declared_functions())


def test_library_has_gfx950_code_object():
    from paper_2412_01138_amd import peifem
    data = open(peifem.LIB_PATH, "rb").read()
    assert b"gfx950" in data


_STRUCTS = [("pe_space_factor", "SpaceFactor"), ("pe_time_factor", "TimeFactor"),
            ("pe_term", "Term"), ("pe_moving_hat", "MovingHat"),
            ("pe_solve_params", "SolveParams"), ("pe_solve_report", "SolveReport"),
            ("pe_kernel_stat", "KernelStat")]


def test_struct_layouts_match_header(tmp_path):
    """Size and field offsets of every struct of the binding equal what a C
    compiler makes of include/peifem.h."""
    import shutil
    import subprocess
    from paper_2412_01138_amd import peifem
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "peifem.h"', "int main(void) {"]
    for cname, pyname in _STRUCTS:
        lines.append(f'printf("{pyname} size %zu\\n", sizeof({cname}));')
        for field, _ in getattr(peifem, pyname)._fields_:
            lines.append(f'printf("{pyname} {field} %zu\\n", offsetof({cname}, {field}));')
    for const in ("PE_K_COUNT", "PE_MAX_ITERS", "PE_MAX_STAGES", "PE_MAX_TERMS", "PE_MAX_DIM",
                  "PE_MLP_PARAMS"):
        lines.append(f'printf("const {const} %d\\n", (int){const});')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        pyname, field, val = line.split()
        if pyname == "const":
            assert getattr(peifem, field) == int(val), (field, val)
            continue
        cls = getattr(peifem, pyname)
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), (pyname, field, got, val)
        seen += 1
    assert seen == sum(1 + len(getattr(peifem, p)._fields_) for _, p in _STRUCTS)
    assert peifem.PE_K_COUNT == len(peifem.KERNEL_CLASSES)


def test_error_path_without_gpu_is_reported():
    """A bad argument is rejected on the host before any device call."""
    from paper_2412_01138_amd import peifem
    L = peifem.load_library()
    h = ctypes.c_void_p()
    n = (ctypes.c_int32 * 1)(0)
    lo = (ctypes.c_double * 1)(0.0)
    hi = (ctypes.c_double * 1)(1.0)
    st = L.pe_init_grid(ctypes.byref(h), 1, n, lo, hi, 1.0, 0, 3, None)
    assert st == peifem.PE_E_ARG
    assert b"n[0]" in L.pe_last_error()
