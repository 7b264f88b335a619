"""Autotuner for the FP32 sweep's length bins.

For every read-length range it times the candidate kernel configurations
(lanes per pair P, rows per lane K with P*K > m) on an equal-length synthetic
batch, kernel time only, and keeps the fastest: the protocol of the paper's
per-length peak measurement (Section IV-B, Fig. 4), used here to fill the
bin table that the plan reads ("max_read_len lanes rows" per line).

    python -m paper_2411_11547_amd.tune [--out FILE] [--hap-len 350] [--pairs 65536]

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


def main():
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
