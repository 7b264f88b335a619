"""ph_forward_batch_noalloc, the forward that allocates nothing, against
ph_forward_batch with a plan built on the same (built-in) bin table: the
same statuses, FP64 values bit for bit and FP32 values to 1e-5 (a plan
sweeps a read against several haplotypes as one chain, which groups the
FP32 partial sums of the row-m sum differently from single pairs), on two
calls in a row that share the library's fixed scratch array, the second
with a smaller input; both also against the FP64 oracle (FP32 pairs to
1e-3, FP64 pairs to 1e-9)."""
import numpy as np
import pytest

from gpu_util import binding, check_against_oracle, oracle, say, wl
from test_gpu_parity import RAGGED_M, RAGGED_N, _ragged

pytestmark = pytest.mark.gpu


def _plan_forward(prob, log10_params=None):
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, tune_table="builtin")
    lp = None if log10_params is None else torch.from_numpy(log10_params).cuda()
    out, st = plan.forward(dev, lp)
    torch.cuda.synchronize()
    res = out.cpu().numpy().copy(), st.cpu().numpy().copy()
    plan.close()
    return res


def _noalloc_forward(prob, log10_params=None):
    import torch
    dev = binding.DeviceProblem(prob)
    lp = None if log10_params is None else torch.from_numpy(log10_params).cuda()
    out, st = binding.forward_noalloc(prob, dev, lp)
    torch.cuda.synchronize()
    return out.cpu().numpy().copy(), st.cpu().numpy().copy()


def _same(prob, a, b):
    (va, sa), (vb, sb) = a, b
    assert np.array_equal(sa, sb), np.nonzero(sa != sb)[0][:10]
    f64 = (sa == binding.PAIR_FP64) | (sa == binding.PAIR_FP64_FLOOR)
    diff = np.nonzero(f64 & (va.view(np.int64) != vb.view(np.int64)))[0]
    assert len(diff) == 0, (diff[:10], va[diff[:10]], vb[diff[:10]])
    err = np.abs(va[~f64] - vb[~f64])
    assert err.size == 0 or err.max() <= 1e-5, err.max()


def test_noalloc_matches_plan_two_calls():
    import torch
    torch.cuda.set_device(0)
    # first call: reads at every bin edge up to 1023, haplotypes with N, and
    # precision-stress pairs that go to both FP64 sweeps
    ms, ns = RAGGED_M, RAGGED_N
    big = _ragged(11, [ms[:9], ms[9:18], ms[18:]], [ns[:6], ns[5:12], ns[11:]])
    rng = np.random.default_rng(11)
    hn = rng.random(len(big.hap_bases)) < 0.03
    big.hap_bases[hn] = 4
    stress = wl.config3(pairs=40)
    say(f"no-alloc call 1: {big.num_pairs} ragged pairs")
    a = _noalloc_forward(big)
    b = _plan_forward(big)
    _same(big, a, b)
    check_against_oracle(big, *a)
    say(f"no-alloc call 2: {stress.num_pairs} precision-stress pairs")
    a = _noalloc_forward(stress)
    assert (a[1] == binding.PAIR_FP64).any()
    _same(stress, a, _plan_forward(stress))
    check_against_oracle(stress, *a)
    # smaller again: the 32 pairs of the 150 bp reference workload
    small = wl.config0()
    say(f"no-alloc call 3: {small.num_pairs} pairs")
    a = _noalloc_forward(small)
    _same(small, a, _plan_forward(small))
    check_against_oracle(small, *a)


def test_noalloc_explicit_params():
    prob = wl.config0()
    rng = np.random.default_rng(3)
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    par *= 10 ** rng.uniform(-0.3, 0.3, par.shape)  # off the Phred manifold
    lp = np.log10(par).astype(np.float32)
    say("no-alloc explicit parameters")
    a = _noalloc_forward(prob, lp)
    _same(prob, a, _plan_forward(prob, lp))
    check_against_oracle(prob, *a, log10_params=lp)
