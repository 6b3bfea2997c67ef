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


def test_struct_sizes_match_header():
    from paper_2412_01138_amd import peifem
    assert ctypes.sizeof(peifem.SpaceFactor) == 5 * 8
    assert ctypes.sizeof(peifem.TimeFactor) == 7 * 8
    assert ctypes.sizeof(peifem.Term) == 8 + 7 * 8 + 3 * 5 * 8
    assert ctypes.sizeof(peifem.SolveReport) == 8 + 64 * 8 + 6 * 8 + 8
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
