"""Build libpairhmm.so for gfx950 with hipcc (in-tree, no JIT cache).

Every HIP source is compiled with packed FP32 instructions disabled
(-target-feature -packed-fp32-ops): the sweep is written as scalar FP32 code
and must stay that way.  IEEE denormals are kept (the hipcc default).

A second library, libpairhmm_ftz.so, differs only in its forward kernels
being built to flush FP32 denormals to zero; it exists so that a test can
show that results above the rescue threshold do not depend on that mode.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpairhmm.so")
LIB_FTZ = os.path.join(HERE, "libpairhmm_ftz.so")
FTZ_SOURCE = "ph_kernels.hip"  # rebuilt with FP32 denormals flushed for LIB_FTZ
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["ph_kernels.hip", "ph_adjoint.hip", "ph_api.cpp", "ph_pipeline.cpp"]
ARCH = os.environ.get("PH_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def _compile(src: str, ftz: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ("_ftz" if ftz else "") + ".o")
    cmd = [hipcc(), *flags()]
    if ftz:
        cmd += ["-fgpu-flush-denormals-to-zero"]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(src, False) for src in SOURCES] + [(FTZ_SOURCE, True)]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        objs = list(ex.map(lambda j: _compile(*j), jobs))
    main = objs[:len(SOURCES)]
    ftz = [objs[-1] if src == FTZ_SOURCE else o for src, o in zip(SOURCES, main)]
    for lib, os_ in ((LIB, main), (LIB_FTZ, ftz)):
        tmp = lib + ".tmp"
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *os_]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"link of {os.path.basename(lib)} failed")
        os.replace(tmp, lib)
        if verbose:
            print(f"built {lib}")
    return LIB


if __name__ == "__main__":
    build()
