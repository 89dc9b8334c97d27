"""Build libtfmm.so in-tree for gfx950 (hipcc for the HIP sources, g++ for host math).

    python -m paper_2010_00520_amd.build        # or paper_2010_00520_amd.build.build()

Always recompiles.  The DFT codelet header is generated first by csrc/gen_dft.py.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtfmm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
NO_PK = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC]
# host code calling the HIP runtime and ROCm libraries (operator setup, solver)
HOST_HIP_UNITS = ("setup_gpu", "solver")
DEVICE_UNITS = ("kernels", "zstage_full", "zstage_tucker", "zstage_tuckerw", "zstage_tt3d", "zstage_tt4d", "noalloc",
                "setup_kernels", "xpass", "farfield")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + os.path.basename(cmd[-1]))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    _run([sys.executable, os.path.join(CSRC, "gen_dft.py"), os.path.join(CSRC, "dft_codelets.h")])
    jobs = [
        ["g++"] + COMMON + ["-pthread", "-c", os.path.join(CSRC, "host_math.cpp"), "-o",
                            os.path.join(BUILD, "host_math.o")],
        [HIPCC, "--offload-arch=" + ARCH] + COMMON + NO_PK + ["-c", os.path.join(CSRC, "api.cpp"), "-o",
                                                             os.path.join(BUILD, "api.o")],
    ] + [
        [HIPCC, "--offload-arch=" + ARCH] + COMMON + NO_PK + ["-c", os.path.join(CSRC, f + ".cpp"), "-o",
                                                             os.path.join(BUILD, f + ".o")]
        for f in HOST_HIP_UNITS
    ] + [
        [HIPCC, "--offload-arch=" + ARCH] + COMMON + NO_PK + ["-c", os.path.join(CSRC, f + ".hip"), "-o",
                                                             os.path.join(BUILD, f + ".o")]
        for f in DEVICE_UNITS
    ]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(_run, jobs))
    objs = [os.path.join(BUILD, n + ".o") for n in ("host_math", "api") + HOST_HIP_UNITS + DEVICE_UNITS]
    tmp = LIB + ".tmp"
    # hipFFT, rocBLAS and rocSOLVER serve the FP64 operator setup and the
    # solver's FP64 vector operations
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs +
         ["-pthread", "-L/opt/rocm/lib", "-lhipfft", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
