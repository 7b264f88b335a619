"""GPU checks of the host-input streaming forward (ph_pipeline_*): results
are identical, pair by pair and bit for bit, to one plan over the device-
resident problem with the same bin table (a pair's sum does not depend on
the tile it shares or on the subset it is in: padding columns add exact
zeros; it does depend on its lane count, which sets how columns fall into
the 64-step partial sums), for several subset sizes, pinned and pageable
inputs, and repeated calls; a sample is checked against the oracle."""
import numpy as np
import pytest

from gpu_util import binding, check_against_oracle, oracle, say, wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    yield


def resident(prob):
    import torch
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    out, st = plan.forward(dev)
    torch.cuda.synchronize()
    res = out.cpu().numpy().copy(), st.cpu().numpy().copy()
    plan.close()
    return res


@pytest.mark.parametrize("cap_frac,pinned,sets", [(0.13, True, 0), (0.13, True, 2), (0.13, True, 3),
                                                 (0.5, False, 0), (0.0, True, 0)])
def test_pipeline_matches_resident_plan(cap_frac, pinned, sets):
    """sets = 0: one buffer set per subset (this problem fits); 2 and 3:
    buffer sets reused in turn, with the copies waiting for compute."""
    prob = wl.config2(regions=40)
    cap = int(prob.total_cells * cap_frac)
    ref, ref_st = resident(prob)
    pipe = binding.Pipeline(prob, max_subset_cells=cap, pinned=pinned, buffer_sets=sets)
    say(f"pipeline: {prob.num_pairs} pairs, {pipe.num_subsets} subsets (cap {cap}), pinned={pinned}, "
        f"buffer sets {sets or 'auto'}")
    if cap_frac > 0:
        assert pipe.num_subsets >= (4 if cap_frac < 0.2 else 2)
    assert pipe.num_pairs == prob.num_pairs and pipe.num_cells == prob.total_cells
    for rep in range(2):
        got, st = pipe.forward()
        assert np.array_equal(got.view(np.int64), ref.view(np.int64)), rep
        assert np.array_equal(st, ref_st)
    ms = pipe.ms()
    say(f"  {ms:.2f} ms host to host, {prob.total_cells / (ms * 1e-3) / 1e9:.1f} GCUPS")
    pipe.close()


def test_pipeline_against_oracle_sample():
    prob = wl.config2(regions=40)
    pipe = binding.Pipeline(prob, max_subset_cells=int(prob.total_cells * 0.2))
    got, st = pipe.forward()
    pipe.close()
    idx = np.sort(np.random.default_rng(12).choice(prob.num_pairs, 400, replace=False))
    check_against_oracle(prob, got, st, pairs=idx)
