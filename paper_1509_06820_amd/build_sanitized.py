"""Build a host-sanitized variant of the C ABI: ``_build_asan/librqrcp_asan.so``.

The host side of every source (argument checks, workspace carving, launch
planning, the batched planner) is compiled with AddressSanitizer and
UndefinedBehaviorSanitizer; the device code is compiled as usual, without
sanitizers.  The library is meant for CPU-side checks of the host logic: it
needs the ASan runtime preloaded (``asan_runtime()``), for example::

    LD_PRELOAD=$(python -c 'from paper_1509_06820_amd import build_sanitized as b; print(b.asan_runtime())') \\
    ASAN_OPTIONS=detect_leaks=0 RQRCP_LIB=paper_1509_06820_amd/_build_asan/librqrcp_asan.so \\
    python -m pytest tests/test_capi_cpu.py

(``RQRCP_LIB`` points the binding at this library instead of librqrcp.so.)
Leak detection stays off because the Python interpreter and the HIP runtime
keep allocations alive until exit.

Usage: ``python -m paper_1509_06820_amd.build_sanitized``.
"""

import concurrent.futures as cf
import os
import subprocess
import sys

from paper_1509_06820_amd import build as _b

OUT = os.path.join(_b.PKG, "_build_asan")
LIB = os.path.join(OUT, "librqrcp_asan.so")
CLANG = os.environ.get("RQ_CLANG", "/opt/rocm/llvm/bin/clang++")

# every sanitizer flag applies to the host compilation only
_HOST_SAN = []
for _f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer"):
    _HOST_SAN += ["-Xarch_host", _f]

FLAGS = [f for f in _b.FLAGS if f != "-O3"] + ["-O1", "-g"] + _HOST_SAN


def asan_runtime():
    """Path of the shared ASan runtime of the ROCm clang (to preload)."""
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                       check=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError(f"ASan runtime not found (clang printed {path!r})")
    return path


def _compile(src):
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    cmd = [_b.HIPCC] + FLAGS + ["-c", os.path.join(_b.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (sanitized) failed on {src}:\n{r.stderr}")
    return obj


def stale():
    """True if the sanitized library is missing or older than a source or header."""
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    for d in (_b.CSRC, _b.INCLUDE):
        for f in os.listdir(d):
            if os.path.getmtime(os.path.join(d, f)) > t:
                return True
    return False


def build_sanitized(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    jobs = min(len(_b.SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, _b.SOURCES))
    tmp = LIB + ".tmp"
    # the objects carry their device code already: a host link suffices
    cmd = [CLANG, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan", "-o", tmp] + objs + [
        "-lamdhip64"] + _b.LIBS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build_sanitized(verbose=True)
    sys.exit(0)
