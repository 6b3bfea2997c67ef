"""Argument checks of the C ABI that run on the host before any device call:
every entry point given a null grid (or model) reports PE_E_ARG with a
message, the size queries return 0, the free calls accept null, and
pe_init_grid rejects each bad parameter by name.  No GPU is needed; the
same tests run under the host-sanitizer build of the library."""
import ctypes
import math

import pytest

from paper_2412_01138_amd import peifem


def _default(t):
    if t in (ctypes.c_double, ctypes.c_float):
        return t(0.0)
    if t in (ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t):
        return t(0)
    return None   # pointers, handles, streams


def _status_calls():
    L = peifem.load_library()
    out = []
    for name in peifem.EXPORTS:
        fn = getattr(L, name)
        if fn.restype is ctypes.c_int32 and name not in ("pe_init_grid", "pe_init_grid_periodic",
                                                          "pe_mlp_create"):
            out.append(name)
    return out


@pytest.mark.parametrize("name", _status_calls())
def test_null_handle_is_rejected(name):
    L = peifem.load_library()
    fn = getattr(L, name)
    st = fn(*[_default(t) for t in fn.argtypes])
    assert st == peifem.PE_E_ARG, (name, st)
    assert L.pe_last_error(), name


def test_size_queries_and_frees_accept_null():
    L = peifem.load_library()
    for name in peifem.EXPORTS:
        fn = getattr(L, name)
        if fn.restype is ctypes.c_size_t:
            assert fn(*[_default(t) for t in fn.argtypes]) == 0, name
    L.pe_free_grid(None)
    L.pe_mlp_free(None)
    assert L.pe_grid_dof(None) <= 0
    assert L.pe_mlp_create(None, None, None) == peifem.PE_E_ARG


def _init(dim=2, n=(7, 9), lo=(0.0, 0.0), hi=(1.0, 1.0), D=1.0, precision=0, quad_q=3,
          periodic=None):
    L = peifem.load_library()
    h = ctypes.c_void_p()
    k = max(dim, 1)
    na = (ctypes.c_int32 * k)(*(list(n) + [1] * k)[:k])
    la = (ctypes.c_double * k)(*(list(lo) + [0.0] * k)[:k])
    ha = (ctypes.c_double * k)(*(list(hi) + [1.0] * k)[:k])
    if periodic is None:
        st = L.pe_init_grid(ctypes.byref(h), dim, na, la, ha, D, precision, quad_q, None)
    else:
        pa = (ctypes.c_int32 * k)(*periodic)
        st = L.pe_init_grid_periodic(ctypes.byref(h), dim, na, la, ha, D, precision, quad_q, pa,
                                     None)
    return st, L.pe_last_error().decode()


@pytest.mark.parametrize("kw, words", [
    (dict(dim=0), "dim"), (dict(dim=4), "dim"),
    (dict(D=0.0), "D"), (dict(D=math.nan), "D"), (dict(D=-1.0), "D"),
    (dict(precision=7), "precision"),
    (dict(quad_q=0), "quad_q"), (dict(quad_q=9), "quad_q"),
    (dict(n=(8192, 9)), "n[0]"), (dict(n=(7, 0)), "n[1]"),
    (dict(hi=(1.0, 0.0)), "hi[1]"), (dict(lo=(2.0, 0.0)), "hi[0]"),
    (dict(n=(100, 9), periodic=(1, 0)), "periodic"),
    (dict(n=(64, 63), periodic=(1, 0), precision=1), "FP64"),
])
def test_init_grid_rejects_bad_parameters(kw, words):
    st, msg = _init(**kw)
    assert st == peifem.PE_E_ARG, (kw, st)
    assert words in msg, (kw, msg)


def test_error_paths_under_host_sanitizers(tmp_path):
    """The checks above and the ABI tests, run again with the library's host
    code built under AddressSanitizer and UndefinedBehaviorSanitizer (any
    report ends the child process with a non-zero status)."""
    import os
    import shutil
    import subprocess

    from conftest import ROOT
    from paper_2412_01138_amd import build_lib
    from paper_2412_01138_amd.sanitize import build_sanitized
    if not os.path.exists(build_lib.HIPCC) or shutil.which("gcc") is None:
        pytest.skip("no HIP compiler")
    out = str(tmp_path / "san")
    build_sanitized.build(out)
    env = dict(os.environ, PEIFEM_LIB=os.path.join(out, "libpeifem.so"),
               ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([os.path.join(out, "pysan"), "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-k", "not sanitizers", os.path.join(ROOT, "tests", "test_host_errors.py"),
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr
