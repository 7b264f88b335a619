"""Pins for the FP64 oracle (CPU only).

The oracle is checked against things other than itself: hand-worked closed
forms of Section II-A's definitions, explicit enumeration of every alignment
path, the ungapped special case (a textbook profile scan), exact power-of-two
scale invariance, the forward = backward total, counting identities of the
posterior expected uses, and central finite differences.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import bruteforce
from paper_2411_11547_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.txt")


def codes(s):
    return np.array([wl.CODE_OF[c] for c in s], np.uint8)


def q20_params(m):
    """Base Q20, ins = del = 45, gcp 10, as in the hand-worked fixture."""
    return oracle.params_from_phred(np.full(m, 20), np.full(m, 45), np.full(m, 45), np.full(m, 10))


def random_params(rng, m, normalised=True):
    if normalised:
        Q = 10 ** -rng.uniform(0.5, 4.0, m)
        delta = 10 ** -rng.uniform(1.0, 4.5, m)
        zeta = 10 ** -rng.uniform(1.0, 4.5, m)
        eps = 10 ** -rng.uniform(0.3, 2.0, m)
        return np.stack([1 - delta - zeta, 1 - eps, delta, eps, zeta, 1 - Q, Q / 3], axis=1)
    # arbitrary positive values: the DP must not rely on any normalisation
    return rng.uniform(0.05, 1.0, (m, 7))


# --- Phred decoding -----------------------------------------------------------
def test_phred_decoding_definition():
    # Phred q means error probability 10^(-q/10): Q10 = 10%, Q20 = 1%, Q30 = 0.1%
    p = oracle.params_from_phred([10, 20, 30], [10, 20, 30], [20, 30, 10], [10, 20, 30])
    assert np.allclose(p[:, 5], [0.9, 0.99, 0.999], rtol=0, atol=1e-15)   # 1 - Q
    assert np.allclose(p[:, 6], [0.1 / 3, 0.01 / 3, 0.001 / 3], rtol=1e-15)  # Q / 3
    assert np.allclose(p[:, 2], [0.1, 0.01, 0.001], rtol=1e-15)          # delta from ins
    assert np.allclose(p[:, 4], [0.01, 0.001, 0.1], rtol=1e-15)          # zeta from del
    assert np.allclose(p[:, 3], [0.1, 0.01, 0.001], rtol=1e-15)          # eps from gcp
    # out-transitions of M and of I/D each sum to one; emissions sum to one
    assert np.allclose(p[:, 0] + p[:, 2] + p[:, 4], 1.0, atol=1e-15)
    assert np.allclose(p[:, 1] + p[:, 3], 1.0, atol=1e-15)
    assert np.allclose(p[:, 5] + 3 * p[:, 6], 1.0, atol=1e-15)


# --- hand-worked closed forms ---------------------------------------------------
def _golden_cases():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            read, hap, val = line.split("\t")[:3]
            out.append((read, hap, float(val)))
    return out


@pytest.mark.parametrize("read,hap,expected", _golden_cases())
def test_hand_worked(read, hap, expected):
    r, h = codes(read), codes(hap)
    p = q20_params(len(r))
    L = 10 ** oracle.forward_pair(r, h, p)
    assert L == pytest.approx(expected, rel=1e-13)
    Lb, _ = bruteforce.likelihood(r, h, p)
    assert Lb == pytest.approx(expected, rel=1e-13)


def test_closed_forms_random_params():
    rng = np.random.default_rng(7)
    for _ in range(20):
        p = random_params(rng, 2, normalised=False)
        # 1 x n: every path is D(0, j-1) -> M(1, j)
        n = int(rng.integers(1, 9))
        h = rng.integers(0, 4, n).astype(np.uint8)
        r = np.array([rng.integers(0, 4)], np.uint8)
        lam = np.where(h == r[0], p[0, 5], p[0, 6])
        assert 10 ** oracle.forward_pair(r, h, p[:1]) == pytest.approx(p[0, 1] / n * lam.sum(), rel=1e-13)
        # 2 x 2, three paths
        r2 = rng.integers(0, 4, 2).astype(np.uint8)
        h2 = rng.integers(0, 4, 2).astype(np.uint8)
        l = lambda i, j: p[i, 5] if r2[i] == h2[j] else p[i, 6]
        want = p[0, 1] / 2 * (p[1, 0] * l(0, 0) * l(1, 1) + p[1, 2] * (l(0, 0) + l(0, 1)))
        assert 10 ** oracle.forward_pair(r2, h2, p) == pytest.approx(want, rel=1e-13)


def closed_3x3(r, h, p):
    """L of a 3 x 3 pair as the sum of its nine paths (written out in
    tests/golden/hand_worked.txt), with per-row parameters p [3, 7] =
    {alpha, beta, delta, eps, zeta, lam_match, lam_mismatch}: the deletion
    path M(1,1)->D(1,2)->M(2,3)->I(3,3) uses zeta_1, beta_2 and delta_3, the
    insertion path M(1,1)->I(2,1)->I(3,1) delta_2 and eps_3."""
    al, be, de, ep, ze = (p[:, c] for c in range(5))
    lam = lambda i, j: p[i - 1, 5] if (r[i - 1] == h[j - 1] or r[i - 1] == 4 or h[j - 1] == 4) else p[i - 1, 6]
    tot = (lam(1, 1) * (al[1] * lam(2, 2) * (al[2] * lam(3, 3) + de[2])
                        + de[1] * (be[2] * lam(3, 2) + ep[2])
                        + ze[0] * be[1] * lam(2, 3) * de[2])
           + lam(1, 2) * (al[1] * lam(2, 3) * de[2] + de[1] * (be[2] * lam(3, 3) + ep[2]))
           + lam(1, 3) * de[1] * ep[2])
    return be[0] / 3 * tot


def test_closed_form_3x3_random_params():
    rng = np.random.default_rng(17)
    for trial in range(40):
        p = random_params(rng, 3, normalised=bool(trial % 2))
        r = rng.integers(0, 5, 3).astype(np.uint8)
        h = rng.integers(0, 5, 3).astype(np.uint8)
        want = closed_3x3(r, h, p)
        assert 10 ** oracle.forward_pair(r, h, p) == pytest.approx(want, rel=1e-13)
        assert bruteforce.likelihood(r, h, p)[0] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("read,hap,expected", [c for c in _golden_cases() if len(c[0]) == 3 and len(c[1]) == 3])
def test_golden_3x3_rows_follow_the_closed_form(read, hap, expected):
    assert closed_3x3(codes(read), codes(hap), q20_params(3)) == pytest.approx(expected, rel=1e-14)


def test_d00_reading_and_single_cell():
    # D(0,0) = 1/n: a 1x1 pair has the single path D(0,0) -> M(1,1)
    p = q20_params(1)
    assert 10 ** oracle.forward_pair(codes("A"), codes("A"), p) == pytest.approx(0.9 * 0.99, rel=1e-15)


# --- brute-force enumeration ----------------------------------------------------
@pytest.mark.parametrize("literal_n", [False, True])
def test_bruteforce_random_tiny(literal_n):
    rng = np.random.default_rng(11 + literal_n)
    for trial in range(60):
        m = int(rng.integers(1, 6))
        n = int(rng.integers(1, 7))
        r = rng.integers(0, 5, m).astype(np.uint8)   # includes N
        h = rng.integers(0, 5, n).astype(np.uint8)
        p = random_params(rng, m, normalised=bool(trial % 2))
        Lb, count = bruteforce.likelihood(r, h, p, literal_n)
        lo = oracle.forward_pair(r, h, p, literal_n=literal_n)
        assert count > 0
        assert 10 ** lo == pytest.approx(Lb, rel=1e-12), (m, n, trial)


def test_path_counts():
    # number of alignment paths is a property of (m, n) only
    p = q20_params(3)
    assert bruteforce.likelihood(codes("ACG"), codes("ACG"), p)[1] == 9
    assert bruteforce.likelihood(codes("AC"), codes("AC"), p[:2])[1] == 3
    assert bruteforce.likelihood(codes("ACG"), codes("ACGT"), p)[1] == 17


# --- N readings -------------------------------------------------------------------
def test_n_wildcard_equals_all_match_row():
    rng = np.random.default_rng(3)
    for _ in range(20):
        m, n = 7, 11
        r = rng.integers(0, 4, m).astype(np.uint8)
        h = rng.integers(0, 4, n).astype(np.uint8)
        i = int(rng.integers(0, m))
        p = random_params(rng, m)
        rN = r.copy(); rN[i] = 4
        # wildcard: an N read base matches every haplotype base
        p_all = p.copy(); p_all[i, 6] = p_all[i, 5]
        assert oracle.forward_pair(rN, h, p) == pytest.approx(oracle.forward_pair(r, h, p_all), abs=1e-13)
        # literal: an N read base matches no A/C/G/T haplotype base
        p_none = p.copy(); p_none[i, 5] = p_none[i, 6]
        assert oracle.forward_pair(rN, h, p, literal_n=True) == pytest.approx(
            oracle.forward_pair(r, h, p_none), abs=1e-13)


# --- textbook special case: no gaps ---------------------------------------------------
def test_ungapped_profile_scan_150x300():
    """delta = zeta = 0, alpha = 1: I and D never fill, and L is the ungapped
    scan (beta_1 / n) * sum over offsets of the product of emissions."""
    rng = np.random.default_rng(5)
    m, n = 150, 300
    r = rng.integers(0, 4, m).astype(np.uint8)
    h = rng.integers(0, 4, n).astype(np.uint8)
    h[40:40 + m] = r  # one strong diagonal
    Q = 10 ** -rng.uniform(1, 4, m)
    p = np.stack([np.ones(m), np.full(m, 0.9), np.zeros(m), np.full(m, 0.1), np.zeros(m), 1 - Q, Q / 3], 1)
    logs = []
    for j0 in range(0, n - m + 1):
        lam = np.where(r == h[j0:j0 + m], p[:, 5], p[:, 6])
        logs.append(np.sum(np.log10(lam)))
    logs = np.array(logs)
    top = logs.max()
    want = math.log10(p[0, 1] / n) + top + math.log10(np.sum(10 ** (logs - top)))
    assert oracle.forward_pair(r, h, p) == pytest.approx(want, abs=1e-11)


# --- range handling -----------------------------------------------------------------
def test_rescaling_is_exact_in_range():
    rng = np.random.default_rng(9)
    for _ in range(10):
        m, n = int(rng.integers(20, 60)), int(rng.integers(30, 120))
        r = rng.integers(0, 5, m).astype(np.uint8)
        h = rng.integers(0, 5, n).astype(np.uint8)
        p = random_params(rng, m)
        a = oracle.forward_pair(r, h, p, rescale=True)
        b = oracle.forward_pair(r, h, p, rescale=False)
        # power-of-two scaling commutes with rounding, so the DP values agree
        # exactly; only the final log10(sum) + e*log10(2) rounds differently
        assert abs(a - b) <= 8 * np.spacing(abs(b))


def test_rescaling_reaches_below_fp64_range():
    # every read base costs at least a factor 0.005 (mismatch 1e-3, gap open
    # 0.005, gap extension 1e-3), so 400 rows give L < 1e-900 < DBL_MIN
    m, n = 400, 420
    r = np.zeros(m, np.uint8)
    h = np.ones(n, np.uint8)  # all mismatches
    p = np.tile([0.99, 0.999, 0.005, 1e-3, 0.005, 0.997, 1e-3], (m, 1))
    lo = oracle.forward_pair(r, h, p)
    assert np.isfinite(lo) and lo < -900
    assert oracle.forward_pair(r, h, p, rescale=False) == -math.inf


# --- backward ---------------------------------------------------------------------
def test_forward_equals_backward_total():
    rng = np.random.default_rng(21)
    for _ in range(10):
        m, n = int(rng.integers(1, 40)), int(rng.integers(1, 80))
        r = rng.integers(0, 5, m).astype(np.uint8)
        h = rng.integers(0, 5, n).astype(np.uint8)
        p = random_params(rng, m, normalised=bool(rng.integers(0, 2)))
        _, lf, lb = oracle.backward_pair(r, h, p)
        assert lf == pytest.approx(oracle.forward_pair(r, h, p), abs=1e-13)
        assert lb == pytest.approx(lf, abs=1e-12)


def test_gradients_match_bruteforce_expected_uses():
    rng = np.random.default_rng(31)
    names = oracle.EXT_CHANNELS
    for trial in range(25):
        m, n = int(rng.integers(1, 5)), int(rng.integers(1, 6))
        r = rng.integers(0, 5, m).astype(np.uint8)
        h = rng.integers(0, 5, n).astype(np.uint8)
        p = random_params(rng, m, normalised=bool(trial % 2))
        g, _, _ = oracle.backward_pair(r, h, p)
        want, _ = bruteforce.expected_uses(r, h, p)
        for i in range(m):
            for c, name in enumerate(names):
                assert g[i, c] == pytest.approx(want[i][name], rel=1e-11, abs=1e-14), (trial, i, name)


def test_gradient_counting_identities():
    rng = np.random.default_rng(41)
    for _ in range(5):
        m, n = int(rng.integers(5, 40)), int(rng.integers(10, 90))
        r = rng.integers(0, 5, m).astype(np.uint8)
        h = rng.integers(0, 5, n).astype(np.uint8)
        g, _, _ = oracle.backward_pair(r, h, random_params(rng, m))
        a, b, d, ei, ed, z, lm, lx = g.T
        # each path has exactly one M-or-I state per row
        assert np.allclose(lm + lx + d + ei, 1.0, atol=1e-12)
        # every M entry uses alpha or beta
        assert np.allclose(a + b, lm + lx, atol=1e-12)
        # every path leaves the initial D row towards M(1, .) using beta_1
        assert b[0] == pytest.approx(1.0, abs=1e-12)
        assert a[0] == 0 and d[0] == 0 and ei[0] == 0
        # D states of the last row reach no end state
        assert z[-1] == 0 and ed[-1] == 0


def test_gradients_central_fd():
    rng = np.random.default_rng(51)
    m, n = 12, 25
    r = rng.integers(0, 5, m).astype(np.uint8)
    h = rng.integers(0, 5, n).astype(np.uint8)
    p = random_params(rng, m)
    g = oracle.ext_to_7(oracle.backward_pair(r, h, p)[0])
    hstep = 1e-5
    for i in range(m):
        for c in range(7):
            up = p.copy(); up[i, c] *= 10 ** hstep
            dn = p.copy(); dn[i, c] *= 10 ** -hstep
            fd = (oracle.forward_pair(r, h, up) - oracle.forward_pair(r, h, dn)) / (2 * hstep)
            assert fd == pytest.approx(g[i, c], abs=1e-7), (i, c)


# --- batch loop ---------------------------------------------------------------------
def test_batch_loop_matches_single_pairs():
    prob = wl.config0()
    out, used = oracle.forward(prob, return_threads=True)
    assert used >= 1 and len(out) == prob.num_pairs == 32
    r_idx, h_idx = prob.pair_index()
    for k in range(prob.num_pairs):
        b, bq, iq, dq, gq = prob.read(r_idx[k])
        p = oracle.params_from_phred(bq, iq, dq, gq)
        assert out[k] == oracle.forward_pair(b, prob.hap(h_idx[k]), p)


def test_batch_log10_params_mode():
    prob = wl.config0()
    r_idx, _ = prob.pair_index()
    par = oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual, prob.gcp_qual)
    lg = np.log10(par).astype(np.float32)
    a = oracle.forward(prob)
    b = oracle.forward(prob, log10_params=lg)
    # float32 log10 parameters round the probabilities at ~1e-7 relative
    assert np.max(np.abs(a - b)) < 1e-4


def test_batch_backward_consistent():
    prob = wl.config0()
    lf, g7, off, gext = oracle.backward(prob, pairs=[0, 5, 31])
    fw = oracle.forward(prob, pairs=[0, 5, 31])
    assert np.allclose(lf, fw, atol=1e-12)
    assert off[-1] == 300 and g7.shape == (300, 7)
    assert np.allclose(g7[:, 5] + g7[:, 6] + gext[:, 2] + gext[:, 3], 1.0, atol=1e-10)


def test_output_order_and_selection():
    prob = wl.from_strings([(["AC", "GT"], ["ACG", "GT", "TTT"]), (["A"], ["A"])])
    assert prob.num_pairs == 7
    r, h = prob.pair_index()
    assert list(r) == [0, 0, 0, 1, 1, 1, 2] and list(h) == [0, 1, 2, 0, 1, 2, 3]
    sub = prob.select_pairs([4, 6])
    assert np.allclose(oracle.forward(sub), oracle.forward(prob)[[4, 6]], atol=0)


# --- Viterbi (max-product) form --------------------------------------------------------
@pytest.mark.parametrize("literal_n", [False, True])
def test_viterbi_equals_bruteforce_best_path(literal_n):
    """The max-product DP equals the largest single-path probability found
    by enumerating every path; and V <= L <= V x (number of paths)."""
    rng = np.random.default_rng(31 + literal_n)
    for trial in range(60):
        m = int(rng.integers(1, 6))
        n = int(rng.integers(1, 7))
        r = rng.integers(0, 5, m).astype(np.uint8)
        h = rng.integers(0, 5, n).astype(np.uint8)
        p = random_params(rng, m, normalised=bool(trial % 2))
        best, trail = bruteforce.best_path(r, h, p, literal_n)
        L, count = bruteforce.likelihood(r, h, p, literal_n)
        v = oracle.viterbi_pair(r, h, p, literal_n=literal_n)
        assert 10 ** v == pytest.approx(best, rel=1e-12), (m, n, trial)
        assert best <= L * (1 + 1e-12) and L <= best * count * (1 + 1e-12)


def test_viterbi_single_path_equals_forward():
    """A 1x1 pair has exactly one path, so its Viterbi score is L."""
    rng = np.random.default_rng(32)
    for _ in range(10):
        p = random_params(rng, 1)
        r, h = rng.integers(0, 5, 1).astype(np.uint8), rng.integers(0, 5, 1).astype(np.uint8)
        assert bruteforce.likelihood(r, h, p)[1] == 1
        assert oracle.viterbi_pair(r, h, p) == pytest.approx(oracle.forward_pair(r, h, p), abs=1e-14)


def test_viterbi_ungapped_max_scan_150x300():
    """delta = zeta = 0, alpha = 1: the best path is the best diagonal,
    (beta_1 / n) x max over offsets of the product of emissions."""
    rng = np.random.default_rng(33)
    m, n = 150, 300
    r = rng.integers(0, 4, m).astype(np.uint8)
    h = rng.integers(0, 4, n).astype(np.uint8)
    h[70:70 + m] = r
    Q = 10 ** -rng.uniform(1, 4, m)
    p = np.stack([np.ones(m), np.full(m, 0.9), np.zeros(m), np.full(m, 0.1), np.zeros(m), 1 - Q, Q / 3], 1)
    logs = [np.sum(np.log10(np.where(r == h[j0:j0 + m], p[:, 5], p[:, 6]))) for j0 in range(n - m + 1)]
    want = math.log10(p[0, 1] / n) + max(logs)
    assert oracle.viterbi_pair(r, h, p) == pytest.approx(want, abs=1e-11)


def test_viterbi_rescaling_and_batch_loop():
    """Row rescaling leaves in-range scores unchanged, and the batch loop
    equals the single-pair calls (Phred and explicit parameters)."""
    prob = wl.config0()
    r_idx, h_idx = prob.pair_index()
    got = oracle.viterbi(prob)
    lg = np.log10(oracle.params_from_phred(prob.base_qual, prob.ins_qual, prob.del_qual,
                                           prob.gcp_qual)).astype(np.float32)
    got_lg = oracle.viterbi(prob, log10_params=lg)
    for k in range(prob.num_pairs):
        rd = prob.read(r_idx[k])
        p = oracle.params_from_phred(rd[1], rd[2], rd[3], rd[4])
        v0 = oracle.viterbi_pair(rd[0], prob.hap(h_idx[k]), p, rescale=False)
        # the rescaled score differs from the plain one only in the final log10 rounding
        assert oracle.viterbi_pair(rd[0], prob.hap(h_idx[k]), p) == pytest.approx(v0, abs=1e-12)
        assert got[k] == oracle.viterbi_pair(rd[0], prob.hap(h_idx[k]), p)
        assert got_lg[k] == pytest.approx(v0, abs=1e-6)
    assert np.all(got <= oracle.forward(prob) + 1e-12)
