"""GPU parity with N (code 4) in the haplotypes.

Eq. (4) runs over the alphabet {A, C, G, T, N} (Section II-A), and the
library reads N on either side as a match.  The other GPU tests put N only
into reads; here the haplotypes carry N too, so that the haplotype-side N
column of every emission table (FP32 and FP64 sweeps, the windowed long-read
sweeps, the max-product sweep and the adjoint) is checked against the
oracle element by element:

* about 3% N at random haplotype positions;
* an all-N haplotype;
* N in the first column, the last column (next to the PAD columns that
  follow a haplotype), and at the chunk edges of the haplotype ring (chunks
  of 32 columns for groups of up to 32 lanes, 64 for 64-lane groups:
  columns 32, 33, 64, 65, 96, 97, 128, 129).

Codes above 4 are read as N by the kernels (ph_validate reports them): a
problem with such codes must give bit-identical results to the same problem
with those codes replaced by 4, which the oracle checks.
"""
import numpy as np
import pytest

from gpu_util import (TOL32, binding, check_against_oracle, check_plain_against_oracle, gpu_forward, oracle, say,
                      wl)

pytestmark = pytest.mark.gpu

EDGE_COLS = (0, 31, 32, 63, 64, 95, 96, 127, 128)  # 0-based: columns 1, 32, 33, 64, 65, 96, 97, 128, 129


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    binding.load()
    yield


def hap_n_problem(seed, lens_m, lens_n, n_rate=0.03, all_n=True):
    """Batches of related reads and haplotypes (haplotypes: mutated copies of
    one reference; reads: error-bearing stretches of them), with N written
    into the haplotypes after the reads were drawn: at rate n_rate, at the
    first and last column and at the ring's chunk edges of every haplotype;
    with all_n every batch gets one more haplotype, 97 bases of N."""
    rng = np.random.default_rng(seed)
    batches = []
    for m_list, n_list in zip(lens_m, lens_n):
        ref = rng.choice(list("ACGT"), size=max(n_list + [1]) + 8)
        haps = []
        for n in n_list:
            h = ref[:n].copy()
            flip = rng.random(n) < 0.02
            h[flip] = rng.choice(list("ACGT"), size=int(flip.sum()))
            haps.append(h)
        reads = []
        for m in m_list:
            h = haps[int(rng.integers(0, len(haps)))]
            s0 = int(rng.integers(0, max(1, len(h) - m + 1)))
            r = np.array((list(h[s0:s0 + m]) + list(rng.choice(list("ACGT"), size=max(0, m - len(h)))))[:m])
            err = rng.random(m) < 0.02
            r[err] = rng.choice(list("ACGTN"), size=int(err.sum()))
            reads.append("".join(r))
        for h in haps:
            n = len(h)
            h[rng.random(n) < n_rate] = "N"
            for c in EDGE_COLS:
                if c < n:
                    h[c] = "N"
            h[n - 1] = "N"
        if all_n:
            haps.append(np.array(["N"] * 97))
        batches.append((reads, ["".join(h) for h in haps]))
    prob = wl.from_strings(batches)
    prob.base_qual[:] = rng.integers(5, 41, size=len(prob.base_qual))
    prob.ins_qual[:] = rng.integers(20, 46, size=len(prob.ins_qual))
    prob.del_qual[:] = rng.integers(20, 46, size=len(prob.del_qual))
    prob.gcp_qual[:] = rng.integers(5, 20, size=len(prob.gcp_qual))
    n_codes = int((prob.hap_bases == 4).sum())
    assert n_codes >= 0.025 * len(prob.hap_bases), n_codes
    return prob


def _lengths_for(P):
    """Read lengths that the lane group size P takes (K up to 16 rows per
    lane, so reads up to 16 P - 1), spread over its K range."""
    top = 16 * P - 1
    ms = sorted({1, 2, P - 1, P, P + 1, 2 * P + 3, top // 2, top - 1, top} & set(range(1, top + 1)))
    return ms


@pytest.mark.parametrize("force_p", [4, 8, 16, 32, 64])
def test_forward_hap_n_every_group_size(force_p):
    """Forward in every lane group size, FP32 and the FP64 rescue (forced for
    every pair), against the oracle."""
    ms = _lengths_for(force_p)
    prob = hap_n_problem(70 + force_p, [ms[::2], ms[1::2]], [[1, 5, 32, 64, 65, 130, 300], [2, 33, 66, 97, 129, 700]])
    say(f"hap N, P={force_p}: {prob.num_pairs} pairs, read lengths {ms}, "
        f"{int((prob.hap_bases == 4).sum())} N of {len(prob.hap_bases)} haplotype bases")
    ref = oracle.forward(prob)
    got, st = gpu_forward(prob, force_p=force_p)
    check_against_oracle(prob, got, st, ref=ref)
    assert (st == binding.PAIR_FP32).sum() >= 8
    got, st = gpu_forward(prob, force_p=force_p, rescue_threshold=float("inf"), use_graph=False)
    assert np.all(st != binding.PAIR_FP32)
    check_against_oracle(prob, got, st, ref=ref)


def test_forward_hap_n_default_bins_single_and_plain():
    """The tuned bins (groups of 4, 8, 16 and 64 lanes), one persistent launch
    over the bins (reads up to 255) and the plain single-bin kernel."""
    ms = [1, 3, 15, 16, 23, 24, 40, 51, 52, 63, 64, 80, 100, 150, 223, 224, 250, 255, 256, 400, 700, 1023]
    prob = hap_n_problem(80, [ms[::2], ms[1::2]], [[1, 33, 64, 65, 129, 333], [3, 32, 96, 128, 250, 900]])
    ref = oracle.forward(prob)
    say(f"hap N, default bins: {prob.num_pairs} pairs")
    for kw in (dict(), dict(use_graph=False)):
        got, st = gpu_forward(prob, **kw)
        check_against_oracle(prob, got, st, ref=ref)
    # the plain kernel has no FP64 rescue: pairs below the FP32 range report status 3
    got, st = gpu_forward(prob, plain=True, use_graph=False)
    check_plain_against_oracle(prob, got, st, ref=ref)
    assert (st == binding.PAIR_FP32).sum() >= 60
    short = hap_n_problem(81, [[1, 2, 20, 47, 48, 100, 255]], [[1, 64, 300]])
    got, st = gpu_forward(short, single_launch=True)
    check_against_oracle(short, got, st)


def test_all_n_haplotype_closed_form():
    """An all-N haplotype makes every cell a match, so L no longer depends on
    the read's bases: reads with the same qualities and different bases give
    the same result (bitwise on the GPU), equal to the oracle's for an all-A
    read against an all-A haplotype of the same length."""
    rng = np.random.default_rng(82)
    m, n = 120, 200
    reads = ["".join(rng.choice(list("ACGTN"), size=m)) for _ in range(4)] + ["A" * m]
    prob = wl.from_strings([(reads, ["N" * n])])
    q = rng.integers(10, 41, size=m).astype(np.uint8)
    prob.base_qual[:] = np.tile(q, len(reads))
    ref_prob = wl.from_strings([(["A" * m], ["A" * n])])
    ref_prob.base_qual[:] = q
    want = oracle.forward(ref_prob)[0]
    for kw in (dict(), dict(force_p=64), dict(rescue_threshold=float("inf"))):
        got, st = gpu_forward(prob, **kw)
        say(f"  all-N haplotype {kw}: {got}, status {st}, oracle {want:.12f}")
        assert np.all(got.view(np.int64) == got[0:1].view(np.int64)), got
        tol = TOL32 if np.all(st == binding.PAIR_FP32) else 1e-9
        assert np.all(np.abs(got - want) <= tol)


def test_viterbi_hap_n():
    """The max-product sweep with N haplotypes: default bins and 64-lane
    groups, and the FP64 rescue forced for every pair."""
    ms = [1, 7, 15, 16, 33, 63, 64, 100, 150, 255, 256, 500, 1023]
    prob = hap_n_problem(83, [ms[::2], ms[1::2]], [[1, 65, 129, 400], [2, 64, 128, 900]])
    ref = oracle.viterbi(prob)
    import torch
    dev = binding.DeviceProblem(prob)
    for kw in (dict(), dict(force_p=64, use_graph=False), dict(rescue_threshold=float("inf"))):
        plan = binding.Plan(prob, **kw)
        v, sv = plan.viterbi(dev)
        torch.cuda.synchronize()
        say(f"hap N, Viterbi {kw}")
        check_against_oracle(prob, v.cpu().numpy(), sv.cpu().numpy(), ref=ref)
        plan.close()


def test_long_reads_hap_n():
    """Reads longer than 1023 bases (windows of 1024 rows with stored boundary
    rows) against haplotypes with N, FP32 and FP64 windows, forward and
    Viterbi."""
    rng = np.random.default_rng(84)
    ref = rng.choice(list("ACGT"), size=3200)
    reads = []
    for m in (1024, 1500, 2049):
        s0 = int(rng.integers(0, 3200 - m))
        r = ref[s0:s0 + m].copy()
        err = rng.random(m) < 0.01
        r[err] = rng.choice(list("ACGTN"), size=int(err.sum()))
        reads.append("".join(r))
    haps = []
    for a, b in ((0, 1100), (200, 3150), (0, 60)):
        h = ref[a:b].copy()
        h[rng.random(len(h)) < 0.03] = "N"
        h[0] = h[-1] = "N"
        h[63:65] = "N"
        haps.append("".join(h))
    prob = wl.from_strings([(reads, haps)])
    prob.base_qual[:] = rng.integers(20, 41, size=len(prob.base_qual))
    prob.ins_qual[:] = rng.integers(40, 46, size=len(prob.ins_qual))
    prob.del_qual[:] = rng.integers(40, 46, size=len(prob.del_qual))
    prob.gcp_qual[:] = 10
    ref_f = oracle.forward(prob)
    say(f"hap N, long reads: log10 L in [{ref_f.min():.1f}, {ref_f.max():.1f}]")
    got, st = gpu_forward(prob)
    check_against_oracle(prob, got, st, ref=ref_f)
    assert (st == binding.PAIR_FP32).sum() >= 2
    got, st = gpu_forward(prob, rescue_threshold=float("inf"))
    check_against_oracle(prob, got, st, ref=ref_f)
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    v, sv = plan.viterbi(dev)
    torch.cuda.synchronize()
    check_against_oracle(prob, v.cpu().numpy(), sv.cpu().numpy(), ref=oracle.viterbi(prob))
    plan.close()


def test_adjoint_hap_n():
    """Gradients with N haplotypes against the oracle's forward-backward:
    reads in 32- and 64-lane adjoint configurations (FP32 pass), and the
    FP64 pass forced for every pair."""
    from test_gpu_adjoint import compare, gpu_grad, oracle_grad
    ms = [1, 2, 31, 32, 63, 64, 100, 127, 150, 159, 160, 200, 255, 300, 319]
    prob = hap_n_problem(85, [ms[::2], ms[1::2]], [[1, 64, 65, 129, 333], [3, 128, 250]])
    lf = oracle.forward(prob)
    u = np.where(lf > -600.0, np.random.default_rng(86).uniform(0.5, 1.5, prob.num_pairs), 0.0)
    say(f"hap N, adjoint: {prob.num_pairs} pairs, {int((lf < -64).sum())} below the FP32 range")
    assert (u > 0).sum() >= 40
    ref, _ = oracle_grad(prob, u)
    got, _ = gpu_grad(prob, u)
    compare(got, ref, "hap N")
    got, _ = gpu_grad(prob, u, rescue_threshold=float("inf"))
    compare(got, ref, "hap N, FP64 forced")


def test_codes_above_4_read_as_n():
    """Haplotype and read codes 5, 9, 200 and 255: every entry point gives
    bit-identical results to the same problem with those codes set to 4, and
    those match the oracle on the problem with N."""
    import torch
    ms = [10, 40, 63, 100, 150, 255, 300, 1200]
    prob_n = hap_n_problem(87, [ms], [[1, 65, 300, 1250]], all_n=False)
    prob_x = hap_n_problem(87, [ms], [[1, 65, 300, 1250]], all_n=False)
    rng = np.random.default_rng(88)
    hn = np.nonzero(prob_n.hap_bases == 4)[0]
    prob_x.hap_bases[hn] = rng.choice(np.array([5, 9, 200, 255], np.uint8), size=len(hn))
    rn = np.nonzero(prob_n.read_bases == 4)[0]
    assert len(rn) >= 4
    prob_x.read_bases[rn] = rng.choice(np.array([5, 9, 200, 255], np.uint8), size=len(rn))
    say(f"codes above 4: {len(hn)} haplotype and {len(rn)} read positions")
    ref = oracle.forward(prob_n)
    for kw in (dict(), dict(force_p=64), dict(rescue_threshold=float("inf"))):
        gn, sn = gpu_forward(prob_n, **kw)
        gx, sx = gpu_forward(prob_x, **kw)
        assert np.array_equal(gn.view(np.int64), gx.view(np.int64)) and np.array_equal(sn, sx), kw
        check_against_oracle(prob_n, gx, sx, ref=ref)
    dn, dx = binding.DeviceProblem(prob_n), binding.DeviceProblem(prob_x)
    pn, px = binding.Plan(prob_n), binding.Plan(prob_x)
    vn, _ = pn.viterbi(dn)
    vx, svx = px.viterbi(dx)
    torch.cuda.synchronize()
    assert np.array_equal(vn.cpu().numpy().view(np.int64), vx.cpu().numpy().view(np.int64))
    check_against_oracle(prob_n, vx.cpu().numpy(), svx.cpu().numpy(), ref=oracle.viterbi(prob_n))
    with pytest.raises(binding.PHError):
        px.validate(dx)
    pn.validate(dn)
    pn.close()
    px.close()
    # the adjoint (reads up to 319 bases)
    from test_gpu_adjoint import compare, gpu_grad, oracle_grad
    keep = [0, 1, 2, 3, 4, 5]
    sub_n = hap_n_problem(89, [[ms[k] for k in keep]], [[1, 65, 300]], all_n=False)
    sub_x = hap_n_problem(89, [[ms[k] for k in keep]], [[1, 65, 300]], all_n=False)
    sub_x.hap_bases[sub_x.hap_bases == 4] = 9
    sub_x.read_bases[sub_x.read_bases == 4] = 255
    u = np.ones(sub_n.num_pairs)
    lf = oracle.forward(sub_n)
    u[lf < -600.0] = 0.0
    gx, _ = gpu_grad(sub_x, u)
    gn, _ = gpu_grad(sub_n, u)
    ref_g, _ = oracle_grad(sub_n, u)
    compare(gx, ref_g, "codes above 4")
    compare(gn, ref_g, "codes as N")
