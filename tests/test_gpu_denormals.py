"""The FP32 denormal mode does not move results above the rescue threshold.

The library keeps IEEE denormals (the hipcc default for gfx950).  The FP32
sweep starts from D(0,j) = 2^120 / n and sends every pair whose scaled sum
falls below 1e-28 (about 2^-93) to the FP64 sweep, so the cells that matter
for a pair finished in FP32 are normal numbers; only cells of negligible
weight can be denormal.  libpairhmm_ftz.so is the same library with the
forward kernels built to flush FP32 denormals to zero: on the 32 pairs of
the 150 bp reference workload and on 8 regions of the uniform batch, its
statuses must be the same and its FP32 results within 1e-6 of the default
build's (the parity bound is 1e-3)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from gpu_util import binding, gpu_forward, say, wl

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FTZ = os.path.join(ROOT, "paper_2411_11547_amd", "libpairhmm_ftz.so")

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
from gpu_util import binding, gpu_forward, wl
assert binding.LIB_PATH.endswith("libpairhmm_ftz.so"), binding.LIB_PATH
out = {}
for name, prob in (("config0", wl.config0()), ("uniform8", wl.config1(regions=8))):
    got, st = gpu_forward(prob)
    out[name] = [got.tolist(), st.tolist()]
print("RESULT " + json.dumps(out))
"""


def test_flush_denormals_build_matches_default():
    assert os.path.exists(FTZ), "build libpairhmm_ftz.so first (paper_2411_11547_amd/build.py)"
    env = dict(os.environ)
    env["PAIRHMM_LIBRARY"] = FTZ
    say("flush-denormals build: forward in a child process")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT ")][-1]
    ftz = json.loads(line[len("RESULT "):])
    for name, prob in (("config0", wl.config0()), ("uniform8", wl.config1(regions=8))):
        got, st = gpu_forward(prob)
        fgot, fst = np.array(ftz[name][0]), np.array(ftz[name][1], np.uint8)
        assert np.array_equal(st, fst), name
        sel = st == binding.PAIR_FP32
        assert sel.sum() >= 30
        d = np.abs(got[sel] - fgot[sel])
        same = int((got[sel].view(np.int64) == fgot[sel].view(np.int64)).sum())
        say(f"  {name}: {int(sel.sum())} FP32 pairs, max |d| {d.max():.2e}, {same} bit-identical")
        assert d.max() <= 1e-6, (name, d.max())
