"""GPU parity of the adjoint sweep: gradients of sum_p u_p log10 L_p with
respect to the log10 parameters of every read base, against the FP64 oracle's
forward-backward and against FP64 central finite differences.

Tolerance: |g - g_ref| <= 1e-3 |g_ref| + 1e-6 elementwise."""
import numpy as np
import pytest

from gpu_util import binding, oracle, say, wl

pytestmark = pytest.mark.gpu
RTOL, ATOL = 1e-3, 1e-6


def oracle_grad(prob, u, log10_params=None):
    """Per read base, sum over the read's pairs of u_p * g_p (oracle)."""
    lf, g7, off, _ = oracle.backward(prob, log10_params=log10_params)
    r_idx, _ = prob.pair_index()
    out = np.zeros((int(prob.read_offset[-1]), 7))
    for k in range(prob.num_pairs):
        a = prob.read_offset[r_idx[k]]
        out[a:a + (off[k + 1] - off[k])] += u[k] * g7[off[k]:off[k + 1]]
    return out, lf


def gpu_grad(prob, u, log10_params=None, **kw):
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, **kw)
    lp = None if log10_params is None else torch.from_numpy(np.ascontiguousarray(log10_params, np.float32)).cuda()
    g = plan.backward(dev, torch.from_numpy(np.ascontiguousarray(u, np.float64)).cuda(), log10_params=lp)
    torch.cuda.synchronize()
    ms = plan.stage_ms()
    res = g.cpu().numpy().astype(np.float64)
    plan.close()
    return res, ms


def compare(got, ref, what):
    err = np.abs(got - ref)
    bad = err > RTOL * np.abs(ref) + ATOL
    rel = float(np.max(err / (np.abs(ref) + ATOL)))
    say(f"  {what}: {got.shape[0]} rows, max rel err {rel:.2e}, violations {int(bad.sum())}")
    assert np.all(np.isfinite(got))
    assert not bad.any(), np.argwhere(bad)[:5]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield


def test_adjoint_config0_phred():
    say("adjoint config0, Phred parameters, u = 1")
    prob = wl.config0()
    u = np.ones(prob.num_pairs)
    ref, _ = oracle_grad(prob, u)
    got, ms = gpu_grad(prob, u)
    compare(got, ref, "config0")


def test_adjoint_shared_reads_weighted():
    """Reads shared by 8 haplotypes: per-base gradients sum u_p-weighted pair
    gradients (config1 shape, 3 regions)."""
    say("adjoint, shared reads, random upstream gradient")
    prob = wl.config1(regions=3)
    u = np.random.default_rng(1).normal(size=prob.num_pairs)
    ref, _ = oracle_grad(prob, u)
    got, _ = gpu_grad(prob, u)
    compare(got, ref, "config1x3")


def ragged_problem():
    """Reads of lengths at every adjoint configuration edge against
    haplotypes of 1..700 bases (prefixes of the reads' reference): many
    pairs are far outside the FP32 range."""
    rng = np.random.default_rng(2)
    reads, haps = [], []
    ref_seq = rng.choice(list("ACGT"), size=700)
    for m in [1, 2, 5, 31, 32, 63, 64, 95, 96, 127, 128, 158, 159, 160, 191, 192, 250, 255, 256, 300, 318, 319]:
        s0 = int(rng.integers(0, 700 - m))
        r = ref_seq[s0:s0 + m].copy()
        err = rng.random(m) < 0.02
        r[err] = rng.choice(list("ACGTN"), size=int(err.sum()))
        reads.append("".join(r))
    for n in [1, 3, 64, 333, 700]:
        haps.append("".join(ref_seq[:n]))
    prob = wl.from_strings([(reads, haps)])
    prob.base_qual[:] = rng.integers(8, 41, size=len(prob.base_qual))
    prob.ins_qual[:] = rng.integers(25, 46, size=len(prob.ins_qual))
    prob.del_qual[:] = rng.integers(25, 46, size=len(prob.del_qual))
    prob.gcp_qual[:] = rng.integers(5, 20, size=len(prob.gcp_qual))
    return prob


# log10 L below which the FP64 adjoint reports NaN (scaled sum under 2^-1000
# with the 2^1020 start: -2020 log10 2 = -608.1); tests keep a margin
FP64_FLOOR_LOG10 = -600.0


def test_adjoint_ragged_lengths():
    """Every pair above the FP64 floor, FP32 and FP64 passes mixed."""
    say("adjoint, read lengths across every configuration, both precisions")
    prob = ragged_problem()
    lf = oracle.forward(prob)
    u = np.where(lf > FP64_FLOOR_LOG10, 1.0, 0.0)
    say(f"  {int((lf < -64).sum())} of {prob.num_pairs} pairs below the FP32 range, "
        f"{int((u == 0).sum())} below the FP64 floor (u = 0)")
    assert (lf < -64).sum() >= 10 and (u == 1).sum() >= 50
    ref, _ = oracle_grad(prob, u)
    got, _ = gpu_grad(prob, u)
    compare(got, ref, "ragged")


def test_adjoint_fp64_forced_every_pair():
    """A rescue threshold of +inf sends every pair to the FP64 pass (all five
    read-length classes of the ragged set)."""
    say("adjoint, FP64 pass forced for every pair")
    prob = ragged_problem()
    lf = oracle.forward(prob)
    u = np.where(lf > FP64_FLOOR_LOG10, np.random.default_rng(7).uniform(0.5, 1.5, prob.num_pairs), 0.0)
    ref, _ = oracle_grad(prob, u)
    got, _ = gpu_grad(prob, u, rescue_threshold=float("inf"))
    compare(got, ref, "fp64 forced")


def test_adjoint_fp64_precision_stress():
    """Pairs of the precision-stress workload (250 bp reads against 1-5 kb
    divergent haplotypes, 30% low-quality reads): most leave the FP32 range."""
    say("adjoint, precision-stress pairs (FP64 pass)")
    full = wl.config3(pairs=2000)
    idx = np.sort(np.random.default_rng(8).choice(full.num_pairs, 48, replace=False))
    prob = full.select_pairs(idx)
    lf = oracle.forward(prob)
    say(f"  log10 L in [{lf.min():.1f}, {lf.max():.1f}], {int((lf < -64).sum())} of 48 below the FP32 range")
    assert (lf < -64).sum() >= 24 and lf.min() > FP64_FLOOR_LOG10
    u = np.random.default_rng(9).normal(size=prob.num_pairs)
    ref, _ = oracle_grad(prob, u)
    got, _ = gpu_grad(prob, u)
    compare(got, ref, "precision stress")


def test_adjoint_fp64_floor_gives_nan():
    """A pair below the FP64 floor yields NaN gradients on its read's rows
    when its upstream gradient is non-zero, and nothing when it is zero."""
    say("adjoint, pair below the FP64 floor")
    read_ok, read_far = "ACGTACGTAC" * 3, "ACGT" * 75   # 300 bases vs a 1-base haplotype
    prob = wl.from_strings([([read_ok], ["ACGTACGTAC" * 4]), ([read_far], ["A"])], gcp_q=30)
    lf = oracle.forward(prob)
    assert lf[0] > -64 and lf[1] < -700, lf
    got, _ = gpu_grad(prob, np.array([1.0, 1.0]))
    assert np.all(np.isfinite(got[:30])) and np.all(np.isnan(got[30:]))
    got0, _ = gpu_grad(prob, np.array([1.0, 0.0]))
    ref, _ = oracle_grad(prob, np.array([1.0, 0.0]))
    compare(got0, ref, "floor, u = 0")


def test_adjoint_explicit_params():
    say("adjoint, explicit log10 parameters off the Phred manifold")
    prob = wl.config4(pairs=40)
    rng = np.random.default_rng(3)
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    par *= 10 ** rng.uniform(-0.1, 0.1, par.shape)  # stays inside the FP32 sweep's range
    lg = np.log10(par).astype(np.float32)
    u = rng.uniform(0.5, 2.0, prob.num_pairs)
    assert np.all(oracle.forward(prob, log10_params=lg) > -60)
    ref, _ = oracle_grad(prob, u, log10_params=lg)
    got, _ = gpu_grad(prob, u, log10_params=lg)
    compare(got, ref, "explicit")


def test_adjoint_config4_full_vs_oracle():
    say("adjoint, config4 full size (10,000 pairs)")
    prob = wl.config4()
    u = np.ones(prob.num_pairs)
    ref, _ = oracle_grad(prob, u)
    got, ms = gpu_grad(prob, u)
    say(f"  adjoint stage {ms[3]:.3f} ms, {prob.total_cells / (ms[3] * 1e-3) / 1e9:.1f} GCUPS")
    compare(got, ref, "config4")


def test_adjoint_vs_central_fd_32_pairs():
    """FP64 central differences of the oracle forward in log10-parameter space
    (h = 1e-5) on 32 pairs sampled with default_rng(4), 6 rows each."""
    say("adjoint vs FP64 central FD, 32 sampled pairs")
    full = wl.config4()
    idx = np.sort(np.random.default_rng(4).choice(full.num_pairs, 32, replace=False))
    prob = full.select_pairs(idx)
    lg = np.log10(oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual))
    lg32 = lg.astype(np.float32)
    got, _ = gpu_grad(prob, np.ones(prob.num_pairs), log10_params=lg32)
    lin = 10.0 ** lg32.astype(np.float64)
    rng = np.random.default_rng(5)
    h = 1e-5
    errs = []
    for k in range(prob.num_pairs):
        a, b = prob.read_offset[k], prob.read_offset[k + 1]
        read, hap = prob.read_bases[a:b], prob.hap(k)
        p0 = lin[a:b]
        for row in rng.choice(b - a, 6, replace=False):
            for c in range(7):
                up = p0.copy(); up[row, c] *= 10 ** h
                dn = p0.copy(); dn[row, c] *= 10 ** -h
                fd = (oracle.forward_pair(read, hap, up) - oracle.forward_pair(read, hap, dn)) / (2 * h)
                g = got[a + row, c]
                errs.append(abs(g - fd) / (abs(fd) + 1e-6))
                assert abs(g - fd) <= 1e-3 * abs(fd) + 2e-6, (k, row, c, g, fd)
    say(f"  {len(errs)} FD checks, max rel err {max(errs):.2e}")


def test_autograd_function_end_to_end():
    """torch.autograd through PairHMMLogLik: loss = sum_p w_p log10 L_p."""
    import torch
    from paper_2411_11547_amd import autograd as ag
    say("torch.autograd.Function end to end")
    prob = wl.config4(pairs=64)
    lg = np.log10(oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual))
    lg32 = lg.astype(np.float32)
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    x = torch.from_numpy(lg32).cuda().requires_grad_(True)
    w = torch.from_numpy(np.random.default_rng(9).uniform(0.5, 1.5, prob.num_pairs)).cuda()
    y = ag.pairhmm_log10_likelihood(x, plan, dev)
    assert y.dtype == torch.float64 and y.shape == (prob.num_pairs,)
    (y * w).sum().backward()
    torch.cuda.synchronize()
    ref_y = oracle.forward(prob, log10_params=lg32)
    assert np.max(np.abs(y.detach().cpu().numpy() - ref_y)) <= 1e-3
    ref_g, _ = oracle_grad(prob, w.cpu().numpy(), log10_params=lg32)
    compare(x.grad.cpu().numpy().astype(np.float64), ref_g, "autograd")
    plan.close()


def test_adjoint_graph_replay_and_eager():
    """The captured backward replayed three times with the upstream gradient
    changed in place between replays (counters and queues are reset by
    kernels inside the graph), each against the oracle; then the eager
    launch sequence on the same buffers."""
    import torch
    say("adjoint graph replays and eager sequence")
    prob = ragged_problem()
    lf = oracle.forward(prob)
    ok = lf > FP64_FLOOR_LOG10
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, use_graph=True)
    u_dev = torch.zeros(prob.num_pairs, dtype=torch.float64, device="cuda")
    g_dev = torch.empty((int(prob.read_offset[-1]), 7), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(11)
    for rep in range(3):
        u = np.where(ok, rng.uniform(0.5, 1.5, prob.num_pairs), 0.0)
        u_dev.copy_(torch.from_numpy(u))
        plan.backward(dev, u_dev, grad_params=g_dev)
        torch.cuda.synchronize()
        ref, _ = oracle_grad(prob, u)
        compare(g_dev.cpu().numpy().astype(np.float64), ref, f"graph replay {rep}")
    plan.close()
    eager = binding.Plan(prob, use_graph=False)
    eager.backward(dev, u_dev, grad_params=g_dev)
    torch.cuda.synchronize()
    compare(g_dev.cpu().numpy().astype(np.float64), ref, "eager")
    eager.close()


def test_adjoint_gap_continuation_zero_rows():
    """Gap-continuation Phred 0 (beta = 0) on rows below the first: the FP32
    adjoint's rescaled insertion state cannot carry them, so those pairs are
    recomputed by the FP64 pass; Phred 1..4 elsewhere (beta down to 0.21)
    stays in FP32.  150-base reads in 32-lane groups, against the oracle."""
    say("adjoint, gap continuation Phred 0")
    prob = wl.config1(regions=2)
    rng = np.random.default_rng(12)
    prob.gcp_qual[:] = rng.integers(1, 5, size=len(prob.gcp_qual))
    for r in range(0, prob.num_reads, 3):  # every third read gets a beta = 0 row
        a, b = prob.read_offset[r], prob.read_offset[r + 1]
        prob.gcp_qual[a + 1 + int(rng.integers(0, b - a - 1))] = 0
    # positive upstream weights: the per-base sums of expected uses do not
    # cancel, so the elementwise bound measures the kernel, not cancellation
    u = rng.uniform(0.5, 1.5, size=prob.num_pairs)
    ref, _ = oracle_grad(prob, u)
    got, _ = gpu_grad(prob, u)
    compare(got, ref, "gcp 0 rows")


def test_adjoint_small_emission_uses_relative():
    """Rows where almost every probable alignment mismatches (a substituted
    base at Q40) have match-emission uses down to about 1e-15, and rows that
    match have mismatch uses that small: each of the two channels is summed
    from same-signed terms, so it must hold to 1e-3 relative with an absolute
    floor of 1e-14 (the general bound's 1e-6 floor would hide a cancellation
    or a rounding residue of the other channel's magnitude)."""
    say("adjoint, emission uses on substituted and matching rows, relative")
    rng = np.random.default_rng(7)
    hap = "".join(rng.choice(list("ACGT"), 300))
    reads = []
    for _ in range(16):
        s0 = int(rng.integers(0, 150))
        r = list(hap[s0:s0 + 150])
        for p in rng.choice(150, 4, replace=False):
            r[p] = rng.choice([c for c in "ACGT" if c != r[p]])
        reads.append("".join(r))
    prob = wl.from_strings([(reads, [hap])], base_q=40)
    u = np.ones(prob.num_pairs)
    ref, _ = oracle_grad(prob, u)
    got, _ = gpu_grad(prob, u)
    compare(got, ref, "substituted rows")
    for ch, name in ((5, "match"), (6, "mismatch")):
        r, g = ref[:, ch], got[:, ch]
        small = r < 1e-4
        err = np.abs(g - r)
        bad = err > 1e-3 * np.abs(r) + 1e-14
        say(f"  {name} uses: {int(small.sum())} rows below 1e-4 (smallest {r.min():.2e}), "
            f"max rel err {float(np.max(err / (np.abs(r) + 1e-14))):.2e}")
        assert small.sum() >= 50
        assert not bad.any(), (name, np.argwhere(bad)[:5].ravel(), r[bad][:5], g[bad][:5])
