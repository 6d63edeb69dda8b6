"""Build the stmg shared library (HIP for gfx950 + host C++) in-tree.

    python -m paper_1911_09548_amd.build      # writes paper_1911_09548_amd/libstmg.so
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libstmg.so")
BUILD_DIR = os.path.join(HERE, "_build")

HOST_SOURCES = ["space.cpp", "ordering.cpp", "factor.cpp"]
HIP_SOURCES = ["kernels.hip", "twogrid.hip", "factor_dev.hip", "solver.cpp", "server.cpp"]  # .cpp here: host code using the HIP runtime


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-Wall", "-Wno-unused-function",
          "-Wno-unused-result"]
# Packed FP32 instructions stay off in device code (known-bad forms on this GPU).
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]
HOST_FLAGS = ["-fopenmp", "-march=x86-64-v3"]


def _compile(src: str, obj: str, hip: bool) -> None:
    cmd = [_hipcc()] + COMMON + (HIP_FLAGS + ["-x", "hip"] if hip else HOST_FLAGS + ["-x", "c++"])
    cmd += ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = []
    for f in HOST_SOURCES:
        jobs.append((os.path.join(CSRC, f), os.path.join(BUILD_DIR, f + ".o"), False))
    for f in HIP_SOURCES:
        jobs.append((os.path.join(CSRC, f), os.path.join(BUILD_DIR, f + ".o"), True))
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(lambda j: _compile(*j), jobs))
    tmp = OUT + ".tmp"
    # rocBLAS (dense triangular solves and symmetric updates of the device
    # factorisation) resolves to the copy the host process has loaded, else
    # to the ROCm installation
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fopenmp", "-o", tmp] + [j[1] for j in jobs]
    cmd += ["-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
