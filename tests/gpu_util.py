"""Helpers shared by the GPU tests (not collected by pytest)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2411_11547_amd import binding  # noqa: E402
from paper_2411_11547_amd import workloads as wl  # noqa: E402

TOL32 = 1e-3   # |delta log10 L| for pairs finished by the FP32 sweep
TOL64 = 1e-9   # |delta log10 L| for pairs recomputed by the FP64 sweep


def say(*a):
    print(*a, flush=True)


def gpu_forward(prob, log10_params=None, **plan_kw):
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, **plan_kw)
    lp = None
    if log10_params is not None:
        lp = torch.from_numpy(np.ascontiguousarray(log10_params, np.float32)).cuda()
    out, st = plan.forward(dev, lp)
    torch.cuda.synchronize()
    res = out.cpu().numpy().copy(), st.cpu().numpy().copy()
    plan.close()
    return res


def check_against_oracle(prob, got, status, ref=None, log10_params=None, pairs=None):
    """Elementwise comparison, FP32 pairs to TOL32 and FP64 pairs to TOL64."""
    if ref is None:
        ref = oracle.forward(prob, log10_params=log10_params, pairs=pairs)
    if pairs is not None:
        got, status = got[pairs], status[pairs]
    err = np.abs(got - ref)
    fin = np.isfinite(ref)
    assert np.all(np.isfinite(got[fin])), "non-finite GPU result where the oracle is finite"
    s32 = status == binding.PAIR_FP32
    s64 = status == binding.PAIR_FP64
    assert np.all(s32 | s64), f"unexpected status values {np.unique(status)}"
    e32 = float(err[s32].max()) if s32.any() else 0.0
    e64 = float(err[s64].max()) if s64.any() else 0.0
    say(f"  pairs={len(ref)} fp32={int(s32.sum())} max|d|={e32:.3e} fp64={int(s64.sum())} max|d|={e64:.3e}")
    assert e32 <= TOL32, e32
    assert e64 <= TOL64, e64
    return err
