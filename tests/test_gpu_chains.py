"""Haplotype chains of the FP32 binned sweep: in groups of 16 or more lanes a
lane group sweeps its read against a run of its batch's haplotypes, one
after the other, clearing its states in the separator columns between them.

Batches are built so that chains form (several reads of one length bin per
batch): chains of haplotypes of different lengths (each with its own edge
value), haplotypes under 64 bases that start chains of their own, N in the
haplotypes, reads unrelated to their haplotypes whose pairs leave the FP32
range inside a chain (FP64 rescue of a chain's pair), every group size of 16
or more lanes, the Viterbi score and explicit parameters, all against the
oracle; and one batch's results bit for bit inside a larger problem, whose
chains are the same."""
import numpy as np
import pytest

from gpu_util import binding, check_against_oracle, gpu_forward, gpu_viterbi, oracle, say, wl
from test_gpu_parity import _ragged

pytestmark = pytest.mark.gpu

# reads: 8 per length, so that every bin of 16, 32 or 64 lanes gets full tiles
READS = [150] * 8 + [100] * 8 + [230] * 8 + [60] * 4
HAPS = [[300, 70, 64, 5, 180, 1000, 120], [64, 65, 63, 400, 90], [250]]


def _chain_problem(seed, related=True):
    prob = _ragged(seed, [READS, READS[::2], READS[1::3]], HAPS, related=related)
    rng = np.random.default_rng(seed + 1)
    hn = rng.random(len(prob.hap_bases)) < 0.03
    prob.hap_bases[hn] = 4
    return prob


@pytest.mark.parametrize("force_p", [0, 16, 32, 64])
def test_chains_forward_against_oracle(force_p):
    prob = _chain_problem(5)
    say(f"chains: {prob.num_pairs} pairs, force_p={force_p}")
    ref = oracle.forward(prob)
    got, st = gpu_forward(prob, force_p=force_p)
    check_against_oracle(prob, got, st, ref=ref)
    got, st = gpu_forward(prob, force_p=force_p, use_graph=False)
    check_against_oracle(prob, got, st, ref=ref)


def test_chains_rescue_and_viterbi():
    """Unrelated reads: most pairs leave the FP32 range and are rescued from
    inside their chains; the max-product score through the same chains."""
    prob = _chain_problem(6, related=False)
    ref = oracle.forward(prob)
    got, st = gpu_forward(prob)
    say(f"chains, unrelated reads: {int((st == binding.PAIR_FP64).sum())} of {prob.num_pairs} pairs rescued")
    assert (st == binding.PAIR_FP64).sum() > prob.num_pairs // 2
    check_against_oracle(prob, got, st, ref=ref)
    rel = _chain_problem(7)
    v, sv = gpu_viterbi(rel)
    check_against_oracle(rel, v, sv, ref=oracle.viterbi(rel))


def test_chains_explicit_params():
    prob = _chain_problem(8)
    rng = np.random.default_rng(9)
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    par *= 10 ** rng.uniform(-0.3, 0.3, par.shape)
    lp = np.log10(par).astype(np.float32)
    got, st = gpu_forward(prob, log10_params=lp)
    check_against_oracle(prob, got, st, log10_params=lp)


def test_chain_results_inside_a_larger_problem():
    """A batch alone and the same batch among others: the same chains, so the
    same values bit for bit."""
    a = _chain_problem(10)
    k = int(a.batch_read_begin[1] - a.batch_read_begin[0]) * int(a.batch_hap_begin[1] - a.batch_hap_begin[0])
    one = _ragged(10, [READS], HAPS[:1])
    one.base_qual[:] = a.base_qual[:len(one.base_qual)]
    one.ins_qual[:] = a.ins_qual[:len(one.ins_qual)]
    one.del_qual[:] = a.del_qual[:len(one.del_qual)]
    one.gcp_qual[:] = a.gcp_qual[:len(one.gcp_qual)]
    one.read_bases[:] = a.read_bases[:len(one.read_bases)]
    one.hap_bases[:] = a.hap_bases[:len(one.hap_bases)]
    ga, sa = gpu_forward(a)
    g1, s1 = gpu_forward(one)
    assert one.num_pairs == k
    assert np.array_equal(sa[:k], s1)
    assert np.array_equal(ga[:k].view(np.int64), g1.view(np.int64))
    check_against_oracle(one, g1, s1)
