"""Build libdwf.so (HIP, gfx950) in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 instruction
selection disabled (-packed-fp32-ops) and linked into one shared library
next to this file.  Run as ``python -m paper_2602_14454_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdwf.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("DWF_OFFLOAD_ARCH", "gfx950")

SOURCES = ["hop.hip", "blas.hip", "fifth_dim.cpp", "objects.cpp", "ops.cpp", "slot_blas.hip", "ptc_kernels.hip", "fgcr_kernels.hip", "gauge.hip", "eo5d.hip", "eo5d_solve.cpp", "solver.cpp", "fgcr.cpp", "ptc.cpp", "batch.cpp", "lanczos.cpp", "api.cpp"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _hip_runtime_dir() -> str:
    """Directory of the HIP runtime the process will use.

    PyTorch-ROCm ships its own libamdhip64.so (soname libamdhip64.so.7).
    libdwf is linked against that file, so its symbol set is checked against
    the runtime torch uses; at load time the Python binding loads torch first,
    and the dynamic loader then binds libdwf's libamdhip64.so.7 dependency to
    torch's already-loaded runtime: one HIP runtime per process, so torch's
    streams and memory are native handles for libdwf.  A C program without
    torch gets /opt/rocm's runtime.
    """
    env = os.environ.get("DWF_HIP_RUNTIME_DIR")
    if env:
        return env
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return "/opt/rocm/lib"


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]


def _compile(src: str, defines=(), build_dir=None) -> str:
    obj = os.path.join(build_dir or BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + _flags() + [f"-D{d}" for d in defines] + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile and link libdwf.so; `defines` are extra -D macros (tuning variants)."""
    bdir = BUILD_DIR if not defines else os.path.join(BUILD_DIR, "v_" + "_".join(d.replace("=", "") for d in defines))
    os.makedirs(bdir, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2) // 2))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, defines, bdir), SOURCES))
    tmp = out + ".tmp"
    rt = _hip_runtime_dir()
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-no-hip-rt", "-o", tmp] + objs + [
        os.path.join(rt, "libamdhip64.so")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
