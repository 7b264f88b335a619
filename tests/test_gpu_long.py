"""GPU parity of reads longer than 1023 bases (windowed sweeps of 1024 rows
with stored boundary rows, FP32 then FP64 for pairs below the FP32 range)
against the FP64 oracle."""
import numpy as np
import pytest

from gpu_util import binding, check_against_oracle, gpu_forward, oracle, say, wl

pytestmark = pytest.mark.gpu

LONG_M = [1024, 1025, 1500, 2047, 2048, 2049, 3000]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield


def long_problem(seed=21):
    """Two batches: long reads (window edges 1024, 2048) and a few short reads
    against haplotypes of 40..3100 bases taken from the reads' reference, so
    that pairs fall in the FP32 range, in the FP64 range and below it."""
    rng = np.random.default_rng(seed)
    ref = rng.choice(list("ACGT"), size=4000)
    reads = []
    for m in LONG_M + [90, 700]:
        s0 = int(rng.integers(0, 4000 - m))
        r = ref[s0:s0 + m].copy()
        err = rng.random(m) < 0.01
        r[err] = rng.choice(list("ACGTN"), size=int(err.sum()))
        reads.append("".join(r))
    haps = ["".join(ref[:n]) for n in (40, 1100)] + ["".join(ref[500:3600])]
    prob = wl.from_strings([(reads[:4], haps), (reads[4:], haps[1:])])
    prob.base_qual[:] = rng.integers(20, 41, size=len(prob.base_qual))
    prob.ins_qual[:] = rng.integers(40, 46, size=len(prob.ins_qual))
    prob.del_qual[:] = rng.integers(40, 46, size=len(prob.del_qual))
    prob.gcp_qual[:] = 10
    return prob


def test_long_reads_against_oracle():
    prob = long_problem()
    say(f"long reads: {prob.num_pairs} pairs, read lengths {sorted(set(prob.read_lengths.tolist()))}")
    got, st = gpu_forward(prob)
    ref = oracle.forward(prob)
    say(f"  statuses {np.bincount(st, minlength=3).tolist()}, log10 L in [{ref.min():.1f}, {ref.max():.1f}]")
    assert (st == binding.PAIR_FP32).sum() >= 6 and (st == binding.PAIR_FP64).sum() >= 3
    check_against_oracle(prob, got, st, ref=ref)


def test_rescued_count_includes_long_pairs():
    """ph_plan_rescued counts every pair sent to an FP64 sweep, those of the
    windowed long-read sweep included, and a ph_validate call after the
    forward leaves that count as it was."""
    import torch
    prob = long_problem()
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    out, st = plan.forward(dev)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    r_idx, _ = prob.pair_index()
    long_pair = prob.read_lengths[r_idx] > 1023
    sent = st != binding.PAIR_FP32
    say(f"  rescued {plan.rescued()}, FP64 statuses {int(sent.sum())} ({int((sent & long_pair).sum())} long)")
    assert (sent & long_pair).sum() >= 2 and (sent & ~long_pair).sum() >= 1
    assert plan.rescued() == int(sent.sum())
    plan.validate(dev)
    assert plan.rescued() == int(sent.sum())
    plan.close()


def test_long_reads_forced_fp64():
    prob = long_problem(seed=22)
    got, st = gpu_forward(prob, rescue_threshold=float("inf"))
    assert np.all(st != binding.PAIR_FP32)
    check_against_oracle(prob, got, st)


def test_long_reads_explicit_params_and_replay():
    import torch
    prob = long_problem(seed=23)
    rng = np.random.default_rng(24)
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    par *= 10 ** rng.uniform(-0.05, 0.05, par.shape)
    lg = np.log10(par).astype(np.float32)
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    x = torch.from_numpy(lg).cuda()
    out1, st1 = plan.forward(dev, log10_params=x)
    torch.cuda.synchronize()
    a1, s1 = out1.cpu().numpy().copy(), st1.cpu().numpy().copy()
    out2, st2 = plan.forward(dev, log10_params=x)
    torch.cuda.synchronize()
    assert np.array_equal(a1.view(np.int64), out2.cpu().numpy().view(np.int64))
    assert np.array_equal(s1, st2.cpu().numpy())
    plan.close()
    check_against_oracle(prob, a1, s1, log10_params=lg)


def test_long_read_row_outside_fp32_states_in_an_earlier_window():
    """An insertion gap-open quality rising from Phred 2 to 90 between rows
    299 and 300 of a long read (kE > 2^20, outside the FP32 states), in its
    first window: the FP32 windowed sweep's final window must still send the
    pair to the FP64 sweep, and no other pair changes status."""
    prob = long_problem()
    got0, st0 = gpu_forward(prob)
    r_idx, _ = prob.pair_index()
    m_all = np.diff(prob.read_offset)
    cand = [r for r in range(prob.num_reads) if m_all[r] > 1024 and np.any(st0[r_idx == r] == binding.PAIR_FP32)]
    assert cand, "no long read with a pair finished in FP32"
    r = cand[0]
    prob.ins_qual[prob.read_offset[r] + 299] = 2
    prob.ins_qual[prob.read_offset[r] + 300] = 90
    mine = r_idx == r
    say(f"long read {r} (m = {m_all[r]}): gap-open Phred 2 -> 90 at row 300, "
        f"{int((st0[mine] == 0).sum())} FP32 pairs before")
    got, st = gpu_forward(prob)
    check_against_oracle(prob, got, st)
    assert np.all(st[mine] != binding.PAIR_FP32)
    assert np.all(st[mine & (st0 == binding.PAIR_FP32)] == binding.PAIR_FP64)
    assert np.array_equal(st[~mine], st0[~mine])


def test_long_read_explicit_alpha_zero_in_an_earlier_window():
    """Explicit parameters with alpha = 0 on row 300 of a long read (the
    FP32 rule evaluated in FP64 by the final window for the rows of earlier
    windows): its pairs go to the FP64 sweep, no other pair changes status,
    and every pair matches the oracle on the same parameters."""
    prob = long_problem(seed=26)
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    lg0 = np.log10(par).astype(np.float32)
    got0, st0 = gpu_forward(prob, log10_params=lg0)
    r_idx, _ = prob.pair_index()
    m_all = np.diff(prob.read_offset)
    cand = [r for r in range(prob.num_reads) if m_all[r] > 1024 and np.any(st0[r_idx == r] == binding.PAIR_FP32)]
    assert cand, "no long read with a pair finished in FP32"
    r = cand[0]
    par[prob.read_offset[r] + 300, 0] = 0.0
    with np.errstate(divide="ignore"):
        lg = np.log10(par).astype(np.float32)
    mine = r_idx == r
    say(f"long read {r} (m = {m_all[r]}): explicit alpha = 0 on row 300, "
        f"{int((st0[mine] == 0).sum())} FP32 pairs before")
    got, st = gpu_forward(prob, log10_params=lg)
    check_against_oracle(prob, got, st, log10_params=lg)
    assert np.all(st[mine] != binding.PAIR_FP32)
    assert np.all(st[mine & (st0 == binding.PAIR_FP32)] == binding.PAIR_FP64)
    assert np.array_equal(st[~mine], st0[~mine])


def test_maximum_read_length():
    """A read of 65,535 bases (the longest the plan takes: 64 windows of 1,024
    rows) against haplotypes of 1,000 and 1,700 bases, in explicit-parameter
    mode with a gap continuation of 1 - 2^-13 (exact in FP32, so that 64,535
    insertion rows do not compound a rounding of the parameter), which keeps
    the likelihood inside the FP32 range; against the oracle."""
    rng = np.random.default_rng(25)
    m = 65535
    hap = rng.choice(list("ACGT"), size=1700)
    read = np.concatenate([hap[:1000], rng.choice(list("ACGT"), size=m - 1000)])
    prob = wl.from_strings([(["".join(read)], ["".join(hap[:1000]), "".join(hap)])])
    par = np.empty((m, 7))
    eps, delta, zeta, q = 1 - 2.0 ** -13, 0.1, 1e-4, 1e-3
    par[:, 0] = 1 - delta - zeta
    par[:, 1] = 1 - eps
    par[:, 2] = delta
    par[:, 3] = eps
    par[:, 4] = zeta
    par[:, 5] = 1 - q
    par[:, 6] = q / 3
    lg = np.log10(par).astype(np.float32)
    say(f"maximum read length {m}: {prob.num_pairs} pairs")
    got, st = gpu_forward(prob, log10_params=lg)
    ref = oracle.forward(prob, log10_params=lg)
    say(f"  log10 L {ref}, statuses {st}")
    assert np.all(np.isfinite(ref))
    check_against_oracle(prob, got, st, ref=ref)
