"""Build the HIP library ``libmpsdmrg.so`` for gfx950 with hipcc.

Usage: ``python -m paper_2207_05612_amd.build`` (or ``build()`` from Python).
Every source is compiled on each call; objects go to ``_build/`` next to this
file and the shared library is written in-tree, next to this file.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD_DIR = os.path.join(HERE, "_build")
LIB_NAME = "libmpsdmrg.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
SOURCES = ["cgemm.hip", "cgemm_bf16.hip", "tensor_ops.hip", "hetrd.hip", "tridiag_dc.hip", "statevector.hip", "driver.cpp"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), res.stderr))
    return obj


# The library must share PyTorch's HIP runtime: two runtimes in one process
# fail on whichever initialises second.  PyTorch ships libamdhip64 / rocBLAS /
# rocSOLVER under torch/lib with the same sonames as /opt/rocm's, so the
# library links through in-tree symlinks (RT_DIR, found at run time via
# $ORIGIN) that point at PyTorch's files; the loader then maps one copy.
RT_DIR = os.path.join(HERE, "_rt")
RT_LIBS = {"libamdhip64.so.7": "libamdhip64.so", "librocsolver.so.0": "librocsolver.so",
           "librocblas.so.5": "librocblas.so"}


def _torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("PyTorch (ROCm build) is required: it provides the HIP runtime")
    return os.path.join(list(spec.submodule_search_locations)[0], "lib")


def _runtime_links() -> None:
    """Mirror torch/lib (shared objects and data directories) into RT_DIR, plus versioned aliases.

    PyTorch's libraries locate their own dependencies through $ORIGIN, which is
    the directory of the path they were opened by; mirroring the whole
    directory keeps every transitive dependency on PyTorch's copy.
    """
    tl = _torch_lib_dir()
    os.makedirs(RT_DIR, exist_ok=True)
    wanted = {}
    for name in os.listdir(tl):
        path = os.path.join(tl, name)
        # shared objects, and data directories that libraries locate next to
        # themselves (rocBLAS reads <its directory>/rocblas/library)
        if (".so" in name and os.path.isfile(path)) or os.path.isdir(path):
            wanted[name] = path
    for link, target in RT_LIBS.items():
        if target not in wanted:
            raise RuntimeError("missing %s in PyTorch's lib directory %s" % (target, tl))
        wanted[link] = wanted[target]
    for link, src in wanted.items():
        dst = os.path.join(RT_DIR, link)
        if os.path.islink(dst) and os.readlink(dst) == src:
            continue
        if os.path.islink(dst) or os.path.exists(dst):
            os.remove(dst)
        os.symlink(src, dst)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    _runtime_links()
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp] + objs + \
          ["-L" + RT_DIR, "-l:librocsolver.so.0", "-l:librocblas.so.5", "-l:libamdhip64.so.7",
           "-Wl,--disable-new-dtags", "-Wl,-rpath,$ORIGIN/_rt", "-Wl,--no-undefined"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), res.stderr))
    os.replace(tmp, LIB_PATH)
    if verbose:
        print("built", LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
