"""Brute-force Pair-HMM likelihood by enumerating every alignment path.

TEST INFRASTRUCTURE ONLY.  Pure Python, for tiny pairs (m, n <= 6).

The forward algorithm sums the probability of every path through the hidden
states (Section II-A).  This module walks those paths one at a time instead
of filling DP matrices, so that a slip in the DP code (a wrong index, a
dropped term, a swapped operand) shows up as a disagreement.

Path semantics read off Eq. (1)-(3) and the initialisation:
* a path starts in the initial D state of row 0 at some column j0 in 0..n,
  with weight 1/n;
* from a state at (i-1, j-1) it may enter M(i, j) with weight
  lam_ij * alpha_i (from M) or lam_ij * beta_i (from I or D);
* from M(i-1, j) it may enter I(i, j) with weight delta_i, from I(i-1, j)
  with weight eps_i;
* from M(i, j-1) it may enter D(i, j) with weight zeta_i, from D(i, j-1)
  with weight eps_i (not in row 0, whose D values are fixed, and not from
  column 0 of rows >= 1, whose values are the zero constants);
* it ends in M(m, j) or I(m, j), j in 1..n, with weight one.
"""
from __future__ import annotations


def _lam(params, i, r, h, j, literal_n):
    ri, hj = r[i - 1], h[j - 1]
    match = (ri == hj) if literal_n else (ri == hj or ri == 4 or hj == 4)
    return params[i - 1][5] if match else params[i - 1][6]


def enumerate_paths(read, hap, params, literal_n=False):
    """Yield (probability, states) for every complete path.
    params: m rows of (alpha, beta, delta, eps, zeta, lam_match, lam_mismatch)."""
    m, n = len(read), len(hap)
    p = [tuple(float(x) for x in row) for row in params]

    def extend(state, i, j, w, trail):
        # end of a path: M or I in the last row
        if i == m and state in ("M", "I"):
            yield w, trail
        # to M(i+1, j+1)
        if i + 1 <= m and j + 1 <= n:
            lam = _lam(p, i + 1, read, hap, j + 1, literal_n)
            tr = p[i][0] if state == "M" else p[i][1]
            yield from extend("M", i + 1, j + 1, w * lam * tr, trail + [("M", i + 1, j + 1)])
        # to I(i+1, j): from M or I only, and I lives in columns >= 1
        if i + 1 <= m and state in ("M", "I") and j >= 1:
            tr = p[i][2] if state == "M" else p[i][3]
            yield from extend("I", i + 1, j, w * tr, trail + [("I", i + 1, j)])
        # to D(i, j+1): from M or D in rows >= 1 only
        if i >= 1 and j + 1 <= n and state in ("M", "D"):
            tr = p[i - 1][4] if state == "M" else p[i - 1][3]
            yield from extend("D", i, j + 1, w * tr, trail + [("D", i, j + 1)])

    for j0 in range(0, n + 1):
        # the initial D(0, j0) can only be left towards M(1, j0 + 1)
        if j0 + 1 > n or m < 1:
            continue
        lam = _lam(p, 1, read, hap, j0 + 1, literal_n)
        w = (1.0 / n) * p[0][1] * lam
        yield from extend("M", 1, j0 + 1, w, [("D0", 0, j0), ("M", 1, j0 + 1)])


def likelihood(read, hap, params, literal_n=False):
    """(L, number of paths with nonzero structural weight)."""
    total, count = 0.0, 0
    for w, _ in enumerate_paths(read, hap, params, literal_n):
        total += w
        count += 1
    return total, count


def best_path(read, hap, params, literal_n=False):
    """(probability of the most probable path, its states): the Viterbi
    score by exhaustive search."""
    best, trail = 0.0, None
    for w, tr in enumerate_paths(read, hap, params, literal_n):
        if w > best:
            best, trail = w, tr
    return best, trail


def expected_uses(read, hap, params, literal_n=False):
    """Posterior expected number of uses of each parameter per read row:
    sum over paths of probability x (times the path uses theta_i) / L.
    Returns a list of m dicts keyed by the extended channel names."""
    m = len(read)
    names = ("alpha", "beta", "delta", "eps_I", "eps_D", "zeta", "lam_match", "lam_mismatch")
    acc = [dict.fromkeys(names, 0.0) for _ in range(m)]
    total = 0.0
    for w, trail in enumerate_paths(read, hap, params, literal_n):
        total += w
        for (s0, i0, j0), (s1, i1, j1) in zip(trail, trail[1:]):
            row = acc[i1 - 1]
            if s1 == "M":
                row["alpha" if s0 == "M" else "beta"] += w
                ri, hj = read[i1 - 1], hap[j1 - 1]
                match = (ri == hj) if literal_n else (ri == hj or ri == 4 or hj == 4)
                row["lam_match" if match else "lam_mismatch"] += w
            elif s1 == "I":
                row["delta" if s0 == "M" else "eps_I"] += w
            elif s1 == "D":
                row["zeta" if s0 == "M" else "eps_D"] += w
    return [{k: v / total for k, v in row.items()} for row in acc], total
