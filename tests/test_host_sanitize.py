"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The FP64 oracle (plain C) is built with gcc and both sanitizers and run
  over single pairs and the threaded batch loops (tests/sanitize/oracle_driver.c).
* The library's host code (plan and pipeline entry points in ph_api.cpp and
  ph_pipeline.cpp, plus the launchers) is built
  with the sanitizers on the host side only (-Xarch_host before each
  -fsanitize=; device code is not instrumented) and driven through the C ABI
  by tests/sanitize/host_driver.c: every argument and shape check, and plan
  and pipeline creation up to the first HIP call, which fails without a GPU,
  so the partly built plan is torn down again under the sanitizers.

Any sanitizer report aborts the program (-fno-sanitize-recover=all), which
fails the test.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
CSRC = os.path.join(ROOT, "paper_2411_11547_amd", "csrc")
LIB_SOURCES = ["ph_kernels.hip", "ph_adjoint.hip", "ph_api.cpp", "ph_pipeline.cpp"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def _env():
    env = dict(os.environ)
    # leak checks stay on; reports abort with a non-zero status
    env["ASAN_OPTIONS"] = "abort_on_error=0:halt_on_error=1:detect_leaks=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.pop("LD_PRELOAD", None)
    return env


def test_oracle_under_asan_ubsan():
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run([cc, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-pthread", "-o", exe, os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "pairhmm_oracle.c"), "-lm"])
    r = _run([exe], env=_env())
    assert "0 mismatches" in r.stdout, r.stdout


def test_host_abi_under_asan_ubsan():
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]

    def comp(src):
        obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
        _run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fPIC",
              "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              *HOST_SAN, *inc, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(len(LIB_SOURCES)) as ex:
        objs = list(ex.map(comp, LIB_SOURCES))
    drv = os.path.join(OUT, "host_driver.o")
    _run([hipcc, "-x", "c", *HOST_SAN, *inc, "-c", os.path.join(HERE, "host_driver.c"), "-o", drv])
    exe = os.path.join(OUT, "host_driver")
    _run([hipcc, "--offload-arch=gfx950", *HOST_SAN, "-o", exe, drv, *objs])
    r = _run([exe], env=_env())
    assert "0 failures" in r.stdout, r.stdout + r.stderr
