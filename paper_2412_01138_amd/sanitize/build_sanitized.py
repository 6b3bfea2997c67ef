"""Host-code sanitizer build: libpeifem.so with its host code compiled under
AddressSanitizer and UndefinedBehaviorSanitizer (device code as in the normal
build), and `pysan`, a Python interpreter with the sanitizer runtimes linked
in, which loads it.

    python -m paper_2412_01138_amd.sanitize.build_sanitized [out_dir [address,undefined]]
    PEIFEM_LIB=<out_dir>/libpeifem.so \\
        ASAN_OPTIONS=detect_leaks=0:alloc_dealloc_mismatch=0 \\
        UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 \\
        <out_dir>/pysan -m pytest tests -x -q

Every `-fsanitize=` flag follows `-Xarch_host`: only the host pass of each
HIP source is instrumented.  Leak detection and the new/delete mismatch
check stay off because they report on the uninstrumented Python and runtime
libraries, not on this code.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import sysconfig
from concurrent.futures import ThreadPoolExecutor

from paper_2412_01138_amd import build_lib

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_SAN = ("address", "undefined")


def host_flags(san):
    flags = ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
    for s in san:
        flags += ["-Xarch_host", f"-fsanitize={s}"]
    if "undefined" in san:
        flags += ["-Xarch_host", "-fno-sanitize-recover=undefined"]
    return flags


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)} failed:\n{r.stderr}")


def build(out: str, san=DEFAULT_SAN) -> None:
    os.makedirs(out, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(build_lib.CSRC, "*.hip")))

    def compile_one(src):
        obj = os.path.join(out, os.path.basename(src).replace(".hip", ".o"))
        _run([build_lib.HIPCC, *build_lib.FLAGS, *host_flags(san), "-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    # the sanitizer runtime comes from the executable (pysan), so the library
    # is linked with its sanitizer symbols left undefined
    _run([build_lib.HIPCC, "-shared", f"--offload-arch={build_lib.ARCH}",
          "-o", os.path.join(out, "libpeifem.so"), *objs])
    inc = sysconfig.get_paths()["include"]
    libdir = sysconfig.get_config_var("LIBDIR")
    ver = sysconfig.get_config_var("LDVERSION")
    clang = os.path.join(os.path.dirname(os.path.realpath(build_lib.HIPCC)), "..", "llvm", "bin",
                         "clang")
    _run([clang, "-O1", "-g", "-fsanitize=" + ",".join(san), "-rdynamic",
          os.path.join(HERE, "pysan.c"), "-I", inc, "-L", libdir, f"-lpython{ver}",
          "-Wl,-rpath," + libdir, "-o", os.path.join(out, "pysan")])
    print(f"built {out}/libpeifem.so and {out}/pysan")


if __name__ == "__main__":
    build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(build_lib.ROOT, "_build", "san"),
          tuple(sys.argv[2].split(",")) if len(sys.argv) > 2 else DEFAULT_SAN)
