"""GPU parity of the HIP forward path against the FP64 oracle.

FP32 results must match within |delta log10 L| <= 1e-3 and FP64-rescued
results within 1e-9.  Every case calls the C ABI through the binding.
"""
import math

import numpy as np
import pytest

from gpu_util import TOL32, TOL64, binding, check_against_oracle, gpu_forward, gpu_viterbi, oracle, say, wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    binding.load()
    yield


def test_config0_binned_graph():
    say("config0 binned, graph")
    prob = wl.config0()
    got, st = gpu_forward(prob)
    check_against_oracle(prob, got, st)
    assert np.all(st == binding.PAIR_FP32)


def test_config0_plain():
    say("config0 plain")
    prob = wl.config0()
    got, st = gpu_forward(prob, plain=True, use_graph=False)
    check_against_oracle(prob, got, st)


@pytest.mark.parametrize("force_p", [16, 32, 64])
def test_lane_groups(force_p):
    say(f"lane groups P={force_p}")
    prob = wl.config0()
    got, st = gpu_forward(prob, force_p=force_p, use_graph=False)
    check_against_oracle(prob, got, st)


@pytest.mark.parametrize("force_p", [4, 8])
def test_small_lane_groups_ragged(force_p):
    """Groups of 4 and 8 lanes share 16-lane DPP rows: a group's first lane
    receives the previous group's last (absorbing) row, whose terms must
    drop out exactly.  Reads of every length the group size supports, mixed
    within tiles, against the oracle; forward and Viterbi."""
    say(f"small lane groups P={force_p}")
    top = 4 * 16 - 1 if force_p == 4 else 8 * 16 - 1
    ms = [m for m in range(1, top + 1) if m % 3 == 1 or m in (force_p - 1, force_p, top)]
    prob = _ragged(31 + force_p, [ms[::2], ms[1::2]], [[1, 7, 64, 65, 200], [3, 129, 300]])
    got, st = gpu_forward(prob, force_p=force_p)
    check_against_oracle(prob, got, st)
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, force_p=force_p)
    v, sv = plan.viterbi(dev)
    torch.cuda.synchronize()
    check_against_oracle(prob, v.cpu().numpy(), sv.cpu().numpy(), ref=oracle.viterbi(prob))
    plan.close()


@pytest.mark.parametrize("force_p", [4, 8, 16, 32, 64])
def test_read_ending_at_haplotype_end(force_p):
    """Reads copied from the end of their haplotype put most of L in the last
    column, and reads of P K - 1 bases put the absorbing row in the group's
    last lane, which must still see column n + 1 (where the rescaled FP32
    states collect the last column).  Odd and even n + P, forward and
    Viterbi, one batch per (K, n) so that tiles hold one haplotype length."""
    say(f"reads at the haplotype end, P={force_p}")
    rng = np.random.default_rng(50 + force_p)
    ks = (4, 6) if force_p == 32 else (2, 3, 5)
    batches = []
    for k in ks:
        m = force_p * k - 1
        for n in (m, m + 3, m + 4, m + 11):
            hap = rng.choice(list("ACGT"), size=n)
            reads = ["".join(hap[n - m:])]
            for _ in range(3):  # the same suffix with a few substitutions
                r = hap[n - m:].copy()
                flip = rng.random(m) < 0.02
                r[flip] = rng.choice(list("ACGT"), size=int(flip.sum()))
                reads.append("".join(r))
            batches.append((reads, ["".join(hap)]))
    prob = wl.from_strings(batches)
    prob.base_qual[:] = rng.integers(10, 41, size=len(prob.base_qual))
    prob.gcp_qual[:] = rng.integers(5, 20, size=len(prob.gcp_qual))
    got, st = gpu_forward(prob, force_p=force_p)
    check_against_oracle(prob, got, st)
    assert np.all(st == binding.PAIR_FP32)
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, force_p=force_p)
    v, sv = plan.viterbi(dev)
    torch.cuda.synchronize()
    check_against_oracle(prob, v.cpu().numpy(), sv.cpu().numpy(), ref=oracle.viterbi(prob))
    plan.close()


def test_result_independent_of_tile_partners():
    """A pair's FP32 result is bit-identical whatever pairs share its tile:
    a second batch of reads of the same lengths against slightly longer
    haplotypes lands in the same bins and haplotype-length buckets, which
    changes the tiles' haplotype lengths and step counts."""
    say("results independent of tile partners")
    rng = np.random.default_rng(60)
    ms, ns1, ns2 = [40, 47, 100, 180, 223], [60, 300], [61, 62, 301, 302, 370]
    ref = rng.choice(list("ACGT"), size=400)
    haps1 = ["".join(ref[:n]) for n in ns1]
    haps2 = ["".join(ref[:n]) for n in ns2]
    reads = []
    for m in ms:
        s0 = int(rng.integers(0, 60 - m + 1)) if m < 60 else int(rng.integers(0, 300 - m + 1))
        r = ref[s0:s0 + m].copy()
        err = rng.random(m) < 0.02
        r[err] = rng.choice(list("ACGT"), size=int(err.sum()))
        reads.append("".join(r))
    a = wl.from_strings([(reads, haps1)])
    b = wl.from_strings([(reads, haps1), (reads, haps2)])
    nb = len(a.base_qual)
    for f in ("base_qual", "ins_qual", "del_qual", "gcp_qual"):
        lo, hi = {"base_qual": (10, 41), "ins_qual": (30, 46), "del_qual": (30, 46), "gcp_qual": (5, 20)}[f]
        q = rng.integers(lo, hi, size=len(getattr(b, f))).astype(np.uint8)
        getattr(b, f)[:] = q
        getattr(a, f)[:] = q[:nb]
    for kw in (dict(), dict(force_p=64)):
        ga, sa = gpu_forward(a, **kw)
        gb, sb = gpu_forward(b, **kw)
        k = a.num_pairs
        assert np.array_equal(sa, sb[:k]) and (sa == binding.PAIR_FP32).sum() >= 6, (sa, sb[:k])
        diff = np.nonzero(ga.view(np.int64) != gb[:k].view(np.int64))[0]
        assert len(diff) == 0, (kw, diff, ga[diff], gb[diff])
    check_against_oracle(b, gb, sb)


def _ragged(seed, lens_m, lens_n, related=True):
    """Batches with the given read and haplotype lengths.  related=True makes
    haplotypes mutated copies of one reference and reads error-bearing
    copies of haplotype stretches (extended with random bases when longer
    than the haplotype), so likelihoods stay in the range real data has."""
    rng = np.random.default_rng(seed)
    batches = []
    for m_list, n_list in zip(lens_m, lens_n):
        ref = rng.choice(list("ACGT"), size=max(n_list + [1]) + 8)
        haps = []
        for n in n_list:
            h = ref[:n].copy() if related else rng.choice(list("ACGT"), size=n)
            flip = rng.random(n) < 0.02
            h[flip] = rng.choice(list("ACGT"), size=int(flip.sum()))
            haps.append(h)
        reads = []
        for m in m_list:
            if related and haps:
                h = haps[int(rng.integers(0, len(haps)))]
                s0 = int(rng.integers(0, max(1, len(h) - m + 1)))
                r = list(h[s0:s0 + m]) + list(rng.choice(list("ACGT"), size=max(0, m - len(h))))
                r = np.array(r[:m])
            else:
                r = rng.choice(list("ACGT"), size=m)
            err = rng.random(m) < 0.02
            r[err] = rng.choice(list("ACGTN"), size=int(err.sum()))
            reads.append("".join(r))
        batches.append((reads, ["".join(h) for h in haps]))
    prob = wl.from_strings(batches)
    prob.base_qual[:] = rng.integers(5, 41, size=len(prob.base_qual))
    prob.ins_qual[:] = rng.integers(20, 46, size=len(prob.ins_qual))
    prob.del_qual[:] = rng.integers(20, 46, size=len(prob.del_qual))
    prob.gcp_qual[:] = rng.integers(5, 20, size=len(prob.gcp_qual))
    return prob


RAGGED_M = [1, 2, 15, 16, 17, 31, 32, 47, 63, 64, 100, 127, 128, 150, 191, 200, 239, 240, 255, 256,
            300, 319, 320, 511, 512, 700, 1023]
RAGGED_N = [1, 2, 3, 31, 32, 33, 63, 64, 65, 95, 96, 97, 127, 128, 129, 300, 1000, 1100]


def test_ragged_lengths_every_bin():
    """Reads at every bin edge (15/16, 31/32, ..., 255/256, 319/320, 1023),
    haplotypes around the ring chunks (32 columns, 64 in 64-lane groups), a
    1x1 pair and empty batches, through the default bins, the eager path and
    64-lane groups."""
    say("ragged lengths")
    ms, ns = RAGGED_M, RAGGED_N
    lens_m = [ms[:9], ms[9:18], ms[18:], [1], [], [5, 7]]
    lens_n = [ns[:6], ns[5:12], ns[11:], [1], [10, 20], []]
    prob = _ragged(1, lens_m, lens_n)
    assert prob.num_pairs == 9 * 6 + 9 * 7 + 9 * 7 + 1
    ref = oracle.forward(prob)
    for kw in (dict(), dict(use_graph=False), dict(force_p=64, use_graph=False)):
        got, st = gpu_forward(prob, **kw)
        check_against_oracle(prob, got, st, ref=ref)


def test_haplotype_length_split_bins(tmp_path):
    """A bin table line may send the pairs of its read range whose haplotype
    reaches a length to a second bin (the committed table: reads 240-255 in
    16 x 16 below 2048 haplotype bases, 64 x 4 from there).  Haplotypes on
    both sides of that edge and of a lower one, through the committed table,
    a table splitting at 256 and the Viterbi score, and batches where one
    side holds only a few pairs."""
    say("haplotype-length split bins")
    ns = [100, 255, 256, 257, 1008, 1023, 1024, 2047, 2048, 2049, 2176]
    prob = _ragged(61, [[240, 247, 255], [250, 200], [255]], [ns[:6], ns[5:], [2048, 2047]])
    ref = oracle.forward(prob)
    split = tmp_path / "split.txt"
    split.write_text("223 16 14\n255 16 16 256 32 8\n1023 64 16\n")
    for kw in (dict(), dict(tune_table=str(split)), dict(tune_table=str(split), use_graph=False)):
        got, st = gpu_forward(prob, **kw)
        check_against_oracle(prob, got, st, ref=ref)
    got, st = gpu_viterbi(prob)
    check_against_oracle(prob, got, st, ref=oracle.viterbi(prob))
    for lens_n in ([[300] * 12 + [2100]] * 2, [[2100] * 12 + [300]] * 2):  # 3 of 39 pairs long, or short
        prob = _ragged(62, [[240, 250], [255]], lens_n)
        got, st = gpu_forward(prob)
        check_against_oracle(prob, got, st, ref=oracle.forward(prob))


def test_gap_continuation_zero_rows():
    """Gap-continuation Phred 0 (eps = 1, beta = 0) on rows below the first,
    and Phred 1..4 on every row of some reads: the FP32 sweep's states divide
    by no beta, so every such pair in the FP32 range finishes in FP32 and
    matches the oracle.  Rows at both ends of the read and inside, in the
    default groups and in 64-lane groups."""
    say("gap continuation Phred 0")
    prob = _ragged(41, [[20, 60, 150, 300, 63], [100, 700, 255, 31]], [[80, 200], [150, 900, 60]])
    rng = np.random.default_rng(42)
    m_all = prob.read_lengths
    zero_rows = {0: [5], 1: [59], 3: [1, 150], 6: [699], 8: [30]}  # read -> rows with Phred 0
    for r, rows in zero_rows.items():
        for i in rows:
            assert 1 <= i < m_all[r]
            prob.gcp_qual[prob.read_offset[r] + i] = 0
    for r in (2, 5):  # Phred 1..4 on every row
        a, b = prob.read_offset[r], prob.read_offset[r + 1]
        prob.gcp_qual[a:b] = rng.integers(1, 5, size=b - a)
    ref = oracle.forward(prob)
    r_idx, _ = prob.pair_index()
    zero = np.isin(r_idx, list(zero_rows))
    inside = ref > -60.0  # well inside the FP32 range (rescue below about -64.1)
    say(f"  {int((zero & inside).sum())} pairs with Phred-0 rows in range")
    assert (zero & inside).sum() >= 6
    for kw in (dict(), dict(force_p=64, use_graph=False)):
        got, st = gpu_forward(prob, **kw)
        check_against_oracle(prob, got, st, ref=ref)
        assert np.all(st[inside] == binding.PAIR_FP32), st[inside]


def test_rows_outside_fp32_states():
    """Rows the FP32 sweep's rescaled states cannot carry send exactly their
    pairs to the FP64 sweep: alpha below 2^-20 (insertion and deletion
    gap-open Phred 3 on one row: alpha = 1 - 2 * 10^-0.3 < 0), and an
    insertion gap-open quality rising from 2 to 90 between two rows (kE =
    eps * delta_{i-1} / delta_i = 0.1 * 10^8.8 > 2^20).  A rise from 2 to 60
    (kE = 10^4.8) stays in FP32.  Rows at both ends of the read and inside,
    in the default groups and in 64-lane groups."""
    say("rows outside the FP32 states")
    prob = _ragged(43, [[20, 60, 150, 120, 63], [100, 90, 255, 31]], [[80, 200], [150, 300, 260]])
    prob.gcp_qual[:] = 10
    m_all = prob.read_lengths
    # read -> rows with ins = del = Phred 3; on the last row, so that L stays
    # positive (a negative alpha on an inner row can make it negative)
    low_alpha = {0: [0], 3: [119], 6: [89]}
    steep = {1: [1], 5: [99], 8: [30]}  # read -> rows i with ins Phred 2 at i-1 and 90 at i
    mild = {2: [100], 7: [254]}         # the same with 60 at i: stays in FP32
    for r, rows in low_alpha.items():
        for i in rows:
            assert 0 <= i < m_all[r]
            prob.ins_qual[prob.read_offset[r] + i] = 3
            prob.del_qual[prob.read_offset[r] + i] = 3
    for table, hi in ((steep, 90), (mild, 60)):
        for r, rows in table.items():
            for i in rows:
                assert 1 <= i < m_all[r]
                prob.ins_qual[prob.read_offset[r] + i - 1] = 2
                prob.ins_qual[prob.read_offset[r] + i] = hi
    ref = oracle.forward(prob)
    assert np.all(np.isfinite(ref))
    r_idx, _ = prob.pair_index()
    # alpha on the read's first row is not divided by (its M term has no alpha)
    flagged = np.isin(r_idx, [3, 6] + list(steep))
    inside = ref > -60.0
    say(f"  {int((flagged & inside).sum())} flagged and {int((~flagged & inside).sum())} other pairs in range")
    assert (flagged & inside).sum() >= 8 and (~flagged & inside).sum() >= 6
    assert (np.isin(r_idx, [3, 6]) & inside).sum() >= 3
    assert (np.isin(r_idx, list(mild)) & inside).sum() >= 2
    assert (np.isin(r_idx, [0]) & inside).sum() >= 1
    for kw in (dict(), dict(force_p=64, use_graph=False), dict(single_launch=True)):
        got, st = gpu_forward(prob, **kw)
        check_against_oracle(prob, got, st, ref=ref)
        assert np.all(st[flagged] != binding.PAIR_FP32), st[flagged]
        assert np.all(st[flagged & inside] == binding.PAIR_FP64), st[flagged & inside]
        assert np.all(st[~flagged & inside] == binding.PAIR_FP32), st[~flagged & inside]
    # plain mode has no rescue: the flagged pairs are reported as unrescued
    # FP32 results, never as good ones; the others match the oracle
    got, st = gpu_forward(prob, plain=True, use_graph=False)
    assert np.all(st[flagged] == binding.PAIR_FP32_UNRESCUED), st[flagged]
    good = ~flagged & inside
    assert np.all(st[good] == binding.PAIR_FP32), st[good]
    assert np.max(np.abs(got[good] - ref[good])) <= TOL32


def test_explicit_rows_outside_fp32_states():
    """Explicit parameters (exponentiated in FP64, the FP32 rule evaluated in
    FP64): alpha = 0 on an inner row, delta falling by 10^-8 from one row to
    the next (kE near 10^8 eps > 2^20), and delta = 0 below a row with delta > 0
    each send exactly their pairs to the FP64 sweep; alpha = 0 on the read's
    first row (its M sum has no alpha) and delta falling by 10^-4 stay in
    FP32.  Against the oracle on the same parameters."""
    say("explicit rows outside the FP32 states")
    prob = _ragged(45, [[20, 60, 150, 120, 63], [100, 90, 255, 31]], [[80, 200], [150, 300, 260]])
    prob.gcp_qual[:] = 10
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    off = prob.read_offset
    par[off[0] + 0, 0] = 0.0        # alpha on the first row: not flagged
    par[off[4] + 40, 0] = 0.0       # alpha = 0 inside: flagged
    par[off[8] + 12, 2] *= 1e-8     # steep fall of delta: flagged
    par[off[1] + 30, 2] = 0.0       # delta = 0: flagged
    par[off[2] + 70, 2] *= 1e-4     # mild fall of delta: not flagged
    with np.errstate(divide="ignore"):
        lg = np.log10(par).astype(np.float32)
    ref = oracle.forward(prob, log10_params=lg)
    assert np.all(np.isfinite(ref))
    r_idx, _ = prob.pair_index()
    flagged = np.isin(r_idx, [4, 8, 1])
    inside = ref > -60.0
    say(f"  {int((flagged & inside).sum())} flagged and {int((~flagged & inside).sum())} other pairs in range")
    assert (flagged & inside).sum() >= 4 and (~flagged & inside).sum() >= 6
    assert (np.isin(r_idx, [0]) & inside).sum() >= 1 and (np.isin(r_idx, [2]) & inside).sum() >= 1
    # default bins: the 20- and 31-base reads run in groups of 4 and 8 lanes
    for kw in (dict(), dict(force_p=64, use_graph=False)):
        got, st = gpu_forward(prob, log10_params=lg, **kw)
        check_against_oracle(prob, got, st, ref=ref, log10_params=lg)
        assert np.all(st[flagged] != binding.PAIR_FP32), st[flagged]
        assert np.all(st[flagged & inside] == binding.PAIR_FP64), st[flagged & inside]
        assert np.all(st[~flagged & inside] == binding.PAIR_FP32), st[~flagged & inside]


def test_fp64_rescaled_and_plain_sweeps():
    """The FP64 rescue runs in two sweeps: the rescaled states (It = I/delta,
    Dh = D/zeta, start scale 2^1000) for pairs that left the FP32 range, then
    the plain states for pairs with a row outside the rescaled states and for
    what the rescaled sweep passes on (a sum outside its range).  Explicit
    parameters whose delta falls by 10^-5.5 on each of twelve consecutive
    rows (kE near 3e4, inside the rescaled states, but It growing by that
    factor per row) and whose eps is near 1, every pair forced into FP64,
    against the oracle; ph_plan_rescued counts every pair once."""
    import torch
    say("FP64 rescaled and plain sweeps")
    prob = _ragged(46, [[40, 90, 150, 255, 300], [63, 120, 200]], [[80, 300, 700], [150, 260]])
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    off = prob.read_offset
    for r in (1, 3, 6):
        a = off[r] + 20
        par[a:a + 12, 2] = 10.0 ** (-1.0 - 5.5 * np.arange(1, 13))  # delta
        par[a:a + 12, 3] = 0.999                                      # eps
        par[a:a + 12, 1] = 1 - 0.999                                  # beta
        par[a:a + 12, 0] = 1 - par[a:a + 12, 2] - par[a:a + 12, 4]    # alpha
    lg = np.log10(par).astype(np.float32)
    ref = oracle.forward(prob, log10_params=lg)
    assert np.all(np.isfinite(ref))
    dev = binding.DeviceProblem(prob)
    x = torch.from_numpy(lg).cuda()
    for kw in (dict(rescue_threshold=math.inf), dict()):
        plan = binding.Plan(prob, **kw)
        out, st = plan.forward(dev, x)
        torch.cuda.synchronize()
        got, st = out.cpu().numpy(), st.cpu().numpy()
        check_against_oracle(prob, got, st, ref=ref, log10_params=lg)
        assert plan.rescued() == int((st != binding.PAIR_FP32).sum()), (plan.rescued(), np.bincount(st))
        if kw:
            assert np.all(st != binding.PAIR_FP32)
        plan.close()


def test_fp64_floor_status():
    """Unrelated 500-1023 base reads against random haplotypes fall below the
    FP64 sweep's range (scaled sum < 2^-1000, log10 L below about -608):
    those pairs and only those are flagged PH_PAIR_FP64_FLOOR; the rest
    stay within tolerance."""
    say("FP64 floor")
    prob = _ragged(2, [[64, 300, 511, 700, 1023]], [[100, 700, 1100]], related=False)
    ref = oracle.forward(prob)
    got, st = gpu_forward(prob)
    assert (ref < -650).any() and (ref > -500).any()
    check_against_oracle(prob, got, st, ref=ref)
    assert (st == binding.PAIR_FP64_FLOOR).any()


@pytest.mark.parametrize("gap", [0.0, 1e-30])
def test_ungapped_closed_form_150x300(gap):
    """Explicit parameters with delta = zeta = 0 and alpha = 1: the result is
    the ungapped scan (beta_1/n) sum over offsets of the emission product.
    delta = 0 is outside the FP32 sweep's states (its I is scaled by
    1/delta), so those pairs finish in FP64.  With delta = zeta = 1e-30 a
    read against the haplotype it was copied into (log10 L near -2) changes
    by about 1e-28 from the closed form and finishes in FP32; against the
    other haplotypes gapped paths dominate, and those pairs are compared with
    the oracle instead."""
    say(f"ungapped closed form, delta = zeta = {gap}")
    rng = np.random.default_rng(7)
    m, n = 150, 300
    reads, haps = [], []
    for _ in range(4):
        r = "".join(rng.choice(list("ACGT"), size=m))
        h = list(rng.choice(list("ACGT"), size=n))
        off = int(rng.integers(0, n - m))
        h[off:off + m] = list(r)
        reads.append(r)
        haps.append("".join(h))
    prob = wl.from_strings([(reads, haps)])
    Q = 10 ** -rng.uniform(1.5, 4, len(prob.read_bases))
    lin = np.stack([np.ones_like(Q), np.full_like(Q, 0.9), np.full_like(Q, gap), np.full_like(Q, 0.1),
                    np.full_like(Q, gap), 1 - Q, Q / 3], 1)
    with np.errstate(divide="ignore"):
        lg = np.log10(lin).astype(np.float32)
    got, st = gpu_forward(prob, log10_params=lg)
    lin32 = 10.0 ** lg.astype(np.float64)
    r_idx, h_idx = prob.pair_index()
    for k in range(prob.num_pairs):
        rb = prob.read(r_idx[k])[0]
        hb = prob.hap(h_idx[k])
        p = lin32[prob.read_offset[r_idx[k]]:prob.read_offset[r_idx[k] + 1]]
        logs = [np.sum(np.log10(np.where(rb == hb[j0:j0 + m], p[:, 5], p[:, 6]))) for j0 in range(n - m + 1)]
        top = max(logs)
        want = math.log10(p[0, 1] / n) + top + math.log10(sum(10 ** (x - top) for x in logs))
        if gap == 0.0:
            # every pair finishes in the FP64 sweep: held to the FP64 bound
            assert st[k] == binding.PAIR_FP64, (k, st[k])
            assert abs(got[k] - want) <= TOL64, (k, got[k], want)
        elif r_idx[k] == h_idx[k]:
            assert want > -10.0
            assert abs(got[k] - want) <= TOL32, (k, got[k], want)
            assert st[k] == binding.PAIR_FP32, (k, st[k], want)
    if gap != 0.0:
        check_against_oracle(prob, got, st, log10_params=lg)


def test_explicit_log10_params():
    say("explicit log10 parameters")
    prob = wl.config0()
    rng = np.random.default_rng(3)
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    par *= 10 ** rng.uniform(-0.3, 0.3, par.shape)  # off the Phred manifold
    lg = np.log10(par).astype(np.float32)
    got, st = gpu_forward(prob, log10_params=lg)
    check_against_oracle(prob, got, st, log10_params=lg)


def test_config1_reduced_all_pairs():
    say("config1, 16 regions, all pairs")
    prob = wl.config1(regions=16)
    got, st = gpu_forward(prob)
    check_against_oracle(prob, got, st)


def test_config2_reduced_all_pairs():
    say("config2, 24 regions, all pairs")
    prob = wl.config2(regions=24)
    got, st = gpu_forward(prob)
    check_against_oracle(prob, got, st)


def test_single_launch_mixed():
    """One persistent FP32 launch over every bin (reads <= 255)."""
    say("single persistent launch, config2 subset")
    prob = wl.config2(regions=24)
    got, st = gpu_forward(prob, single_launch=True)
    check_against_oracle(prob, got, st)
    short = _ragged(3, [[1, 2, 20, 47, 48, 100, 255]], [[1, 64, 300]])
    got, st = gpu_forward(short, single_launch=True)
    check_against_oracle(short, got, st)


def test_config1_full_size_sampled():
    """512,000 pairs in the launch configuration the benchmark times; 1,500
    sampled outputs checked one by one against the oracle."""
    say("config1 full size, sampled")
    prob = wl.config1()
    got, st = gpu_forward(prob)
    assert np.all(np.isfinite(got))
    idx = np.random.default_rng(11).choice(prob.num_pairs, 1500, replace=False)
    check_against_oracle(prob, got, st, pairs=idx)


def test_config2_full_size_sampled():
    """The benchmark's mixed batch at full size (2,000 regions, 3,757,266
    pairs) through the default plan (autotuned bins, per-bin launches, graph),
    2,000 seeded sampled pairs checked one by one against the oracle."""
    say("config2 full size, sampled")
    prob = wl.config2()
    got, st = gpu_forward(prob)
    idx = np.sort(np.random.default_rng(7).choice(prob.num_pairs, 2000, replace=False))
    check_against_oracle(prob, got, st, pairs=idx)
    assert np.all(st == binding.PAIR_FP32)


def test_config3_full_size_sampled():
    """The precision-stress set at full size (50,000 pairs, 250 bp reads with
    N bases and low qualities against 1,000-5,000 bp divergent haplotypes):
    most pairs take the FP64 rescue; 400 seeded sampled pairs of each path
    checked against the oracle."""
    say("config3 full size, sampled")
    prob = wl.config3()
    got, st = gpu_forward(prob)
    rng = np.random.default_rng(8)
    idx = []
    for code in (binding.PAIR_FP32, binding.PAIR_FP64):
        cand = np.nonzero(st == code)[0]
        assert len(cand) >= 400, (code, len(cand))
        idx.append(rng.choice(cand, 400, replace=False))
    check_against_oracle(prob, got, st, pairs=np.sort(np.concatenate(idx)))


def test_rescue_path_config3_subset():
    say("config3 subset: FP32 + FP64 rescue")
    prob = wl.config3(pairs=300)
    got, st = gpu_forward(prob)
    err = check_against_oracle(prob, got, st)
    assert (st == binding.PAIR_FP64).any(), "precision stress should send some pairs to FP64"


def test_forced_rescue_all_fp64():
    say("forced rescue: every pair in FP64")
    prob = _ragged(5, [[1, 40, 150, 250, 300, 600]], [[1, 70, 400, 700]])
    got, st = gpu_forward(prob, rescue_threshold=math.inf)
    assert np.all((st == binding.PAIR_FP64) | (st == binding.PAIR_FP64_FLOOR))
    check_against_oracle(prob, got, st)


def test_graph_replay_bitwise():
    """Replays of the captured graph, with other GPU work in between, give
    bitwise-identical results."""
    import torch
    say("graph replay")
    prob = wl.config2(regions=6)
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    outs = []
    for i in range(3):
        out, st = plan.forward(dev)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy().copy())
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    plan.close()
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    eager, _ = gpu_forward(prob, use_graph=False)
    assert np.array_equal(outs[0], eager)


def test_validate_rejects_bad_codes():
    import torch
    say("validate")
    prob = wl.config0()
    prob.hap_bases[7] = 9
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    with pytest.raises(binding.PHError) as e:
        plan.validate(dev)
    assert e.value.status == -1
    prob.hap_bases[7] = 2
    dev2 = binding.DeviceProblem(prob)
    plan.validate(dev2)
    plan.close()


def test_plan_mismatch():
    say("plan mismatch")
    a, b = wl.config0(), wl.config1(regions=1)
    plan = binding.Plan(a)
    dev = binding.DeviceProblem(b)
    with pytest.raises(binding.PHError) as e:
        plan.forward(dev)
    assert e.value.status == -5
    plan.close()
