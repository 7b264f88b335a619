"""Autotuner for the FP32 sweep's length bins.

Stage 1 (sweep): for every read-length range it times the candidate kernel
configurations (lanes per pair P, rows per lane K with P*K > m) on an
equal-length synthetic batch, kernel time only, and keeps the fastest: the
protocol of the paper's per-length peak measurement (Section IV-B, Fig. 4),
used here to fill the bin table that the plan reads ("max_read_len lanes
rows" per line).

Stage 2 (refine): equal-length batches do not see what a mixed batch does
(bins running concurrently, tiles of different haplotype lengths, the tail
of each bin), so the table is then refined on the workload it serves:
range by range, in order of that workload's cells, each of the next-best
configurations of stage 1 replaces the current one, the FP32 sweep stage of
the whole workload is timed, and the change is kept when it is faster by
more than the noise margin.

    python -m paper_2411_11547_amd.tune [--out FILE] [--hap-len 350] [--pairs 65536]
    python -m paper_2411_11547_amd.tune refine [--table FILE] [--out FILE] [--workload 2]

Runs on the GPU; the result for this chip is committed as tune_gfx950.txt.
"""
from __future__ import annotations

import argparse
import os
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tune_gfx950.txt")

# compiled FP32 sweep configurations (mirror of the kernel's instance list)
CONFIGS = [(4, k) for k in range(2, 17)] + [(8, k) for k in range(2, 17)] + \
          [(16, k) for k in range(1, 17)] + [(32, k) for k in (4, 6, 8, 10, 12, 16)] + \
          [(64, k) for k in range(2, 17)]


def ranges():
    """Read-length ranges of the table, aligned with P*K - 1: 4-row steps to
    63, 8-row steps to 127, 16-row steps to 255, then 64-row steps to 1023."""
    out = [(max(1, 4 * k), 4 * k + 3) for k in range(16)]
    out += [(8 * k, 8 * k + 7) for k in range(8, 16)]
    out += [(16 * k, 16 * k + 15) for k in range(8, 16)]
    out += [(64 * k, 64 * k + 63) for k in range(4, 16)]
    return out


def equal_length_problem(m, n, pairs, seed=0):
    """`pairs` independent pairs of read length m and haplotype length n,
    grouped 8 haplotypes per read like the uniform workload."""
    from . import workloads as wl
    rng = np.random.default_rng(seed)
    H = 8
    reads = pairs // H
    ref = wl.random_bases(rng, n + m)
    haps = np.stack([wl.substitute(rng, ref[:n], 0.01) for _ in range(H)])
    rstart = rng.integers(0, max(1, n - m + 1), size=reads)
    idx = rstart[:, None] + np.arange(m)[None, :]
    rb = wl.substitute(rng, ref[np.minimum(idx, n + m - 1)].reshape(-1), 0.01)
    q = wl.illumina_quals(rng, rb.size)
    iq = rng.integers(40, 46, size=rb.size).astype(np.uint8)
    dq = rng.integers(40, 46, size=rb.size).astype(np.uint8)
    gq = np.full(rb.size, 10, np.uint8)
    nb = reads
    return wl.Problem(np.arange(nb + 1), np.arange(nb + 1) * H,
                      np.arange(reads + 1, dtype=np.int64) * m, rb, q, iq, dq, gq,
                      np.arange(reads * H + 1, dtype=np.int64) * n,
                      np.tile(haps.reshape(-1), reads), name=f"tune-{m}x{n}")


def time_config(prob, dev, m, P, K, steps=3):
    import torch
    from . import binding
    with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as f:
        f.write(f"{m} {P} {K}\n")
        path = f.name
    try:
        plan = binding.Plan(prob, tune_table=path, rescue_threshold=1e-300)
        plan.forward(dev)
        torch.cuda.synchronize()
        ms = []
        for _ in range(steps):
            plan.forward(dev)
            ms.append(plan.stage_ms()[1])
        plan.close()
    finally:
        os.unlink(path)
    return float(np.median(ms))


def read_table(path):
    """[(max_m, P, K, alternatives, line, split)] from a table file;
    alternatives are the stage-1 (GCUPS, P, K) entries of the line's comment,
    best first; split is the line's haplotype-length split "n_split P2 K2"
    (pairs of the range with haplotypes of at least n_split bases go to a bin
    of P2 x K2), kept as written, or ""."""
    rows = []
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            body, _, comment = line.partition("#")
            nums = [int(x) for x in body.split()]
            m, P, K = nums[:3]
            split = " ".join(str(x) for x in nums[3:6])
            alts = []
            for tok in comment.split():
                if "x" in tok and ":" in tok:
                    pk, g = tok.split(":")
                    p, k = pk.split("x")
                    alts.append((float(g), int(p), int(k)))
            rows.append([m, P, K, sorted(alts, reverse=True), line.rstrip("\n"), split])
    return rows


def write_table(rows, path, header):
    with open(path, "w") as f:
        f.write("\n".join(header) + "\n")
        for m, P, K, alts, line, split in rows:
            desc = " ".join(f"{p}x{k}:{g:.0f}" for g, p, k in alts)
            f.write(f"{m} {P} {K}{' ' + split if split else ''}  # {desc}\n")


def time_table(rows, prob, dev, steps):
    """Median FP32 sweep stage (ms) of the whole workload under a table."""
    import torch
    from . import binding
    with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as f:
        f.write("".join(f"{m} {P} {K} {split}\n" for m, P, K, _, _, split in rows))
        path = f.name
    try:
        plan = binding.Plan(prob, tune_table=path)
        out = torch.empty(max(plan.num_pairs, 1), dtype=torch.float64, device="cuda")
        st = torch.empty(max(plan.num_pairs, 1), dtype=torch.uint8, device="cuda")
        plan.forward(dev, out=out, status=st)
        torch.cuda.synchronize()
        ms = []
        for _ in range(steps):
            plan.forward(dev, out=out, status=st)
            ms.append(plan.stage_ms()[1])
        plan.close()
    finally:
        os.unlink(path)
    return float(np.median(ms))


def refine(argv):
    ap = argparse.ArgumentParser(prog="tune refine")
    ap.add_argument("--table", default=DEFAULT_TABLE)
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--workload", type=int, default=2, help="workload index (2 = the mixed-length batch)")
    ap.add_argument("--steps", type=int, default=7)
    ap.add_argument("--margin", type=float, default=0.004, help="relative gain a change must exceed")
    ap.add_argument("--alternatives", type=int, default=3)
    ap.add_argument("--min-share", type=float, default=0.005, help="skip ranges with fewer of the cells")
    args = ap.parse_args(argv)
    import torch
    from . import binding, workloads as wl
    assert torch.cuda.is_available()
    binding.load()
    rows = read_table(args.table)
    prob = wl.make(args.workload)
    dev = binding.DeviceProblem(prob)
    r_idx, _ = prob.pair_index()
    m_pair = prob.read_lengths[r_idx]
    cells = prob.pair_cells()
    lo = 1
    share = []
    for i, row in enumerate(rows):
        sel = (m_pair >= lo) & (m_pair <= row[0])
        share.append((float(cells[sel].sum()) / float(cells.sum()), i))
        lo = row[0] + 1
    base = time_table(rows, prob, dev, args.steps)
    print(f"refine on {prob.name}: start {base:.3f} ms", flush=True)
    for frac, i in sorted(share, reverse=True):
        if frac < args.min_share:
            continue
        cur = (rows[i][1], rows[i][2])
        for g, P, K in rows[i][3][:args.alternatives]:
            if (P, K) == cur:
                continue
            trial = [list(r) for r in rows]
            trial[i][1], trial[i][2] = P, K
            ms = time_table(trial, prob, dev, args.steps)
            again = time_table(rows, prob, dev, args.steps)  # the current table, re-timed beside it
            keep = ms < again * (1 - args.margin)
            print(f"  reads <= {rows[i][0]} ({frac:.1%} of cells): {cur[0]}x{cur[1]} {again:.3f} ms, "
                  f"{P}x{K} {ms:.3f} ms{'  kept' if keep else ''}", flush=True)
            base = ms if keep else again
            if keep:
                rows[i][1], rows[i][2] = P, K
                cur = (P, K)
    header = ["# FP32 sweep bin table for gfx950: max_read_len lanes rows_per_lane",
              "# stage 1: equal-length batches (haplotype 350, 65536 pairs), kernel time; the comment of",
              "# each line lists the GCUPS of every configuration tried there",
              f"# stage 2: refined on {prob.name} (FP32 sweep stage of the whole batch, median of {args.steps})"]
    write_table(rows, args.out, header)
    print(f"wrote {args.out}: {base:.3f} ms", flush=True)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "refine":
        return refine(sys.argv[2:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--hap-len", type=int, default=350)
    ap.add_argument("--pairs", type=int, default=65536)
    ap.add_argument("--candidates", type=int, default=2, help="K values tried per lane count")
    args = ap.parse_args()
    import torch
    from . import binding
    assert torch.cuda.is_available()
    binding.load()
    lines = ["# FP32 sweep bin table for gfx950: max_read_len lanes rows_per_lane",
             f"# equal-length batches, haplotype length {args.hap_len}, {args.pairs} pairs, kernel time",
             "# columns after '#' on each line: GCUPS of the chosen and of every tried configuration"]
    for lo, hi in ranges():
        prob = equal_length_problem(hi, args.hap_len, args.pairs)
        dev = binding.DeviceProblem(prob)
        tried = []
        for P in (4, 8, 16, 32, 64):
            ks = sorted(k for (p, k) in CONFIGS if p == P and P * k - 1 >= hi)[:args.candidates]
            for K in ks:
                ms = time_config(prob, dev, hi, P, K)
                tried.append((prob.total_cells / (ms * 1e-3) / 1e9, P, K))
        best = max(tried)
        desc = " ".join(f"{P}x{K}:{g:.0f}" for g, P, K in tried)
        lines.append(f"{hi} {best[1]} {best[2]}  # {best[0]:.0f} GCUPS; {desc}")
        print(lines[-1], flush=True)
        del dev
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
