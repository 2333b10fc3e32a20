"""Build the gfx950 shared library ``lib/libietidp.so`` in-tree with hipcc.

Usage: ``python -m paper_2501_04340_amd.build`` (or ``build()`` from Python).
Every call recompiles all sources.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libietidp.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = [
    os.path.join(CSRC, "api.cpp"),
    os.path.join(CSRC, "nn_api.cpp"),
    os.path.join(CSRC, "host", "mesh_topology.cpp"),
    os.path.join(CSRC, "host", "assemble.cpp"),
    os.path.join(CSRC, "host", "plan.cpp"),
    os.path.join(CSRC, "host", "batch.cpp"),
    os.path.join(CSRC, "host", "partition_check.cpp"),
    os.path.join(CSRC, "device", "kernels.hip"),
    os.path.join(CSRC, "device", "nn_kernels.hip"),
]

ARCH = "gfx950"
COMPILE_TIMEOUT_S = 600
COMMON = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fopenmp",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the library needs the ROCm toolchain")
    return exe


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.relpath(src, CSRC).replace(os.sep, "_") + ".o")
    cmd = [_hipcc(), *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-xhip")
    try:
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=COMPILE_TIMEOUT_S)
    except subprocess.TimeoutExpired:
        raise RuntimeError(f"compilation of {src} exceeded {COMPILE_TIMEOUT_S}s") from None
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"compilation of {src} failed:\n{out}")
    if verbose and out.strip():
        print(out)
    return obj


def _runtime_dirs():
    """Directories searched for the HIP runtime at load time.

    PyTorch ships its own HIP runtime and loads it by path; two runtimes in
    one process cannot share the device, so the library resolves
    libamdhip64 from torch's directory first when torch is installed.
    """
    dirs = []
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            tl = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(tl, "libamdhip64.so")):
                dirs.append(tl)
    except Exception:
        pass
    return dirs + ["/opt/rocm/lib", "/opt/rocm/llvm/lib"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    rpath = ":".join(_runtime_dirs())
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-fopenmp", "-shared", "-o", tmp, *objs,
           "-Wl,--disable-new-dtags", f"-Wl,-rpath,{rpath}", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
