"""GPU parity of the Viterbi score (ph_viterbi_batch: the max-product form
of the same sweep, FP32 with FP64 rescue, windowed for long reads) against
the FP64 oracle's max-product DP; the same tolerances as the forward."""
import numpy as np
import pytest

from gpu_util import binding, check_against_oracle, gpu_viterbi, oracle, say, wl
from test_gpu_long import long_problem
from test_gpu_parity import RAGGED_M, RAGGED_N, _ragged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield


def test_viterbi_config0():
    say("viterbi config0")
    prob = wl.config0()
    got, st = gpu_viterbi(prob)
    check_against_oracle(prob, got, st, ref=oracle.viterbi(prob))


def test_viterbi_ragged_every_bin():
    say("viterbi ragged lengths")
    ms, ns = RAGGED_M, RAGGED_N
    prob = _ragged(1, [ms[:9], ms[9:18], ms[18:], [1], [], [5, 7]],
                   [ns[:6], ns[5:12], ns[11:], [1], [10, 20], []])
    ref = oracle.viterbi(prob)
    for kw in (dict(), dict(use_graph=False), dict(force_p=64, use_graph=False), dict(single_launch=True)):
        got, st = gpu_viterbi(prob, **kw)
        check_against_oracle(prob, got, st, ref=ref)


def test_viterbi_rescue_and_long_reads():
    say("viterbi precision-stress subset and long reads")
    full = wl.config3(pairs=2000)
    idx = np.sort(np.random.default_rng(41).choice(full.num_pairs, 120, replace=False))
    prob = full.select_pairs(idx)
    got, st = gpu_viterbi(prob)
    assert (st == binding.PAIR_FP64).sum() > 20
    check_against_oracle(prob, got, st, ref=oracle.viterbi(prob))
    prob = long_problem(seed=25)
    got, st = gpu_viterbi(prob)
    check_against_oracle(prob, got, st, ref=oracle.viterbi(prob))


def test_viterbi_explicit_params_bounded_by_forward_and_graphs():
    """Explicit parameters; V <= L for every pair; the forward's and the
    Viterbi's stage graphs replayed alternately give the same results."""
    import torch
    prob = wl.config2(regions=30)
    rng = np.random.default_rng(42)
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    par *= 10 ** rng.uniform(-0.1, 0.1, par.shape)
    lg = np.log10(par).astype(np.float32)
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    x = torch.from_numpy(lg).cuda()
    v1, sv1 = (a.cpu().numpy().copy() for a in plan.viterbi(dev, x))
    f1, sf1 = (a.cpu().numpy().copy() for a in plan.forward(dev, x))
    v2, _ = (a.cpu().numpy().copy() for a in plan.viterbi(dev, x))
    f2, _ = (a.cpu().numpy().copy() for a in plan.forward(dev, x))
    torch.cuda.synchronize()
    plan.close()
    assert np.array_equal(v1.view(np.int64), v2.view(np.int64))
    assert np.array_equal(f1.view(np.int64), f2.view(np.int64))
    ok = (sv1 != binding.PAIR_FP64_FLOOR) & (sf1 != binding.PAIR_FP64_FLOOR)
    assert np.all(v1[ok] <= f1[ok] + 1e-3)
    sample = np.sort(rng.choice(prob.num_pairs, 300, replace=False))
    ref = oracle.viterbi(prob, log10_params=lg, pairs=sample)
    check_against_oracle(prob, v1, sv1, ref=ref, pairs=sample)


def test_viterbi_rows_outside_fp32_states():
    """The max-product sweep shares the forward's FP32 rule: rows with alpha
    below 2^-20 (gap-open Phred 3 on insertion and deletion) or a gap-open
    quality rising from Phred 2 to 90 send exactly their pairs to the FP64
    sweep; gap-continuation Phred 0 rows (beta = 0) stay in FP32.  Default
    bins (groups of 4, 8 and 16 lanes) and 64-lane groups."""
    say("viterbi rows outside the FP32 states")
    prob = _ragged(47, [[20, 60, 150, 120, 63], [100, 90, 255, 31]], [[80, 200], [150, 300, 260]])
    prob.gcp_qual[:] = 10
    off = prob.read_offset
    for r, i in ((3, 119), (6, 89)):        # alpha < 0 on the last row
        prob.ins_qual[off[r] + i] = 3
        prob.del_qual[off[r] + i] = 3
    for r, i in ((1, 1), (8, 30)):          # steep rise of the insertion gap-open quality
        prob.ins_qual[off[r] + i - 1] = 2
        prob.ins_qual[off[r] + i] = 90
    prob.gcp_qual[off[4] + 10] = 0          # beta = 0: stays in FP32
    prob.gcp_qual[off[0] + 5] = 0
    ref = oracle.viterbi(prob)
    assert np.all(np.isfinite(ref))
    r_idx, _ = prob.pair_index()
    flagged = np.isin(r_idx, [3, 6, 1, 8])
    inside = ref > -60.0
    say(f"  {int((flagged & inside).sum())} flagged and {int((~flagged & inside).sum())} other pairs in range")
    assert (flagged & inside).sum() >= 4 and (~flagged & inside).sum() >= 4
    assert (np.isin(r_idx, [0, 4]) & inside).sum() >= 2
    for kw in (dict(), dict(force_p=64, use_graph=False)):
        got, st = gpu_viterbi(prob, **kw)
        check_against_oracle(prob, got, st, ref=ref)
        assert np.all(st[flagged] != binding.PAIR_FP32), st[flagged]
        assert np.all(st[flagged & inside] == binding.PAIR_FP64), st[flagged & inside]
        assert np.all(st[~flagged & inside] == binding.PAIR_FP32), st[~flagged & inside]


def test_small_groups_next_to_rows_outside_fp32_states():
    """Groups of 4 lanes: reads of 15 bases fill a 4 x 4 group, so a pair's
    absorbing row is its group's last row, which the next group's first lane
    receives through the lane shift.  Every other read has gap-open Phred 3
    on its last row (alpha < 0, outside the FP32 states): those pairs go to
    the FP64 sweep, and their neighbours in the same waves still finish in
    FP32 and match the oracle, for the Viterbi score and the forward."""
    from gpu_util import gpu_forward
    say("groups of 4 lanes next to pairs outside the FP32 states")
    prob = _ragged(49, [[15] * 12 + [14, 13]], [[40, 50, 60]])
    prob.gcp_qual[:] = 10
    off = prob.read_offset
    flagged_reads = list(range(0, 12, 2))
    for r in flagged_reads:
        prob.ins_qual[off[r] + 14] = 3
        prob.del_qual[off[r] + 14] = 3
    r_idx, _ = prob.pair_index()
    flagged = np.isin(r_idx, flagged_reads)
    for run, ref in ((gpu_viterbi, oracle.viterbi(prob)), (gpu_forward, oracle.forward(prob))):
        assert np.all(np.isfinite(ref))
        inside = ref > -60.0
        assert (flagged & inside).sum() >= 6 and (~flagged & inside).sum() >= 6
        got, st = run(prob)
        check_against_oracle(prob, got, st, ref=ref)
        assert np.all(st[flagged & inside] == binding.PAIR_FP64), st[flagged & inside]
        assert np.all(st[~flagged & inside] == binding.PAIR_FP32), st[~flagged & inside]
