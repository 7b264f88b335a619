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


def gpu_viterbi(prob, log10_params=None, **plan_kw):
    """The max-product score through a plan (ph_viterbi_batch)."""
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, **plan_kw)
    lp = None if log10_params is None else torch.from_numpy(np.ascontiguousarray(log10_params, np.float32)).cuda()
    out, st = plan.viterbi(dev, lp)
    torch.cuda.synchronize()
    res = out.cpu().numpy().copy(), st.cpu().numpy().copy()
    plan.close()
    return res


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


FLOOR_LOG10 = -608.0  # FP64 sweep range floor: scaled sum 2^-1000 at scale 2^1020


def check_against_oracle(prob, got, status, ref=None, log10_params=None, pairs=None):
    """Elementwise comparison: FP32 pairs to TOL32, FP64 pairs to TOL64.
    Pairs below the FP64 sweep's range must carry the floor status (and only
    those); their value is not compared."""
    if ref is None:
        ref = oracle.forward(prob, log10_params=log10_params, pairs=pairs)
    if pairs is not None:
        got, status = got[pairs], status[pairs]
    s32 = status == binding.PAIR_FP32
    s64 = status == binding.PAIR_FP64
    s2 = status == binding.PAIR_FP64_FLOOR
    assert np.all(s32 | s64 | s2), f"unexpected status values {np.unique(status)}"
    assert np.all(ref[s2] < FLOOR_LOG10 + 8), "floor status on a pair inside the FP64 range"
    assert np.all(s2[ref < FLOOR_LOG10 - 12]), "pair below the FP64 range without the floor status"
    cmp = s32 | s64
    assert np.all(np.isfinite(got[cmp])), "non-finite GPU result where a value is expected"
    err = np.abs(got - ref)
    e32 = float(err[s32].max()) if s32.any() else 0.0
    e64 = float(err[s64].max()) if s64.any() else 0.0
    say(f"  pairs={len(ref)} fp32={int(s32.sum())} max|d|={e32:.3e} fp64={int(s64.sum())} "
        f"max|d|={e64:.3e} floor={int(s2.sum())}")
    assert e32 <= TOL32, e32
    assert e64 <= TOL64, e64
    return err


# FP32 sweep range: scaled sum 1e-28 at the start scale 2^120
THRESHOLD_LOG10 = -28.0 - 120 * 0.30102999566398119521


def check_plain_against_oracle(prob, got, status, ref=None):
    """The plain single-bin kernel has no rescue: pairs inside the FP32 range
    (status 0) are compared to TOL32; the others carry status 3, and the
    oracle puts exactly those below the range threshold (within TOL32)."""
    if ref is None:
        ref = oracle.forward(prob)
    s32 = status == binding.PAIR_FP32
    s3 = status == binding.PAIR_FP32_UNRESCUED
    assert np.all(s32 | s3), f"unexpected status values {np.unique(status)}"
    assert np.all(ref[s3] < THRESHOLD_LOG10 + TOL32), "unrescued status on a pair inside the FP32 range"
    assert np.all(ref[s32] > THRESHOLD_LOG10 - TOL32), "FP32 status on a pair below the FP32 range"
    e32 = float(np.abs(got[s32] - ref[s32]).max()) if s32.any() else 0.0
    say(f"  plain: pairs={len(ref)} fp32={int(s32.sum())} max|d|={e32:.3e} unrescued={int(s3.sum())}")
    assert e32 <= TOL32, e32
