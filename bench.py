"""Benchmark: Pair-HMM forward GCUPS on one MI355X.

One step = one forward call over the whole batch: on-device binning, the
FP32 sweeps of every length bin and the FP64 recomputation of pairs below
the FP32 underflow threshold, replayed from a HIP graph, inputs already in
HBM.  GCUPS = sum over pairs of m*n / time / 1e9 (the paper's CUPS, Eq. (5)).

Printed as one JSON line: the binned throughput (value), the plain
single-bin FP32 kernel on the same batch, the FP32 sweep stage against the
FP32 vector roofline, and the FP64 CPU oracle timed on a bounded sample of
the same pairs on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Forward GCUPS on 1 MI355X (binned FP32+FP64 rescue vs plain); adjoint GCUPS"
FLOPS_PER_CELL = 11            # Eq. (1)-(3): 7 multiplications + 4 additions
# FP32 issue slots per cell of the rescaled-state sweep: 4 FMA + 1 MUL, where on gfx950 an FP32 FMA
# issues 16 lanes per clock per SIMD and an FP32 multiply 32 (measured with a microkernel of independent
# chains), so the multiply takes half an FMA slot
FMA_SLOTS_PER_CELL = 4.5
VITERBI_VALU_PER_CELL = 8      # the max-product cell: 5 MUL + 3 MAX
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector peak
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector peak
PEAK_FMA_LANE_OPS = 256 * 4 * 16 * 2.4e9  # unpacked FP32 FMA: CUs x SIMDs x lanes/clk x clock


# HBM traffic of the FP32 sweep stage, from the committed rocprofv3 counter
# summary; reported only while the forward kernel sources and the bin table
# are the ones the counters were taken on
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "fwd32_hbm_traffic_mixed-2000regions.txt")
FORWARD_SOURCES = ("paper_2411_11547_amd/csrc/ph_kernels.hip", "paper_2411_11547_amd/csrc/ph_device.h",
                   "paper_2411_11547_amd/csrc/ph_internal.h", "paper_2411_11547_amd/tune_gfx950.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_tokens(text):
    """C++ source with comments removed and whitespace collapsed, so that the
    hash below changes with the code and not with its comments.  (String and
    character literals in the kernel sources hold no comment markers.)"""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def forward_sources_sha256():
    """Hash of the forward sweep's code (comments and layout ignored): the
    HBM traffic measured for one version is reported only for that version."""
    import hashlib
    h = hashlib.sha256()
    for rel in FORWARD_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_tokens(f.read()).encode())
    return h.hexdigest()


def measured_traffic(workload_name):
    """(bytes per FP32 sweep stage, note) from the counter summary, or None
    when it is missing, for another workload or for other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("workload") != workload_name or kv.get("forward_sources_sha256") != forward_sources_sha256():
        return None
    return float(kv["traffic_bytes_per_launch"])


def workload(cfg: int):
    from paper_2411_11547_amd import workloads as wl
    return wl.make(cfg)


def time_forward_fn(fn, plan, steps, warmup):
    """Like time_forward for any plan call (the Viterbi score); `fn` writes
    into fixed buffers so that the captured graphs are replayed."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
        stages.append(plan.stage_ms())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, np.array(stages)


def time_forward(plan, dev, steps, warmup, stage=True):
    """Seconds per forward call and the per-call stage times; the outputs go
    to the same buffers every call, so the captured stage graphs replay."""
    import torch
    out = torch.empty(max(plan.num_pairs, 1), dtype=torch.float64, device="cuda")
    status = torch.empty(max(plan.num_pairs, 1), dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        plan.forward(dev, out=out, status=status)
    torch.cuda.synchronize()
    stages = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward(dev, out=out, status=status)
        if stage:
            stages.append(plan.stage_ms())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, np.array(stages) if stages else None


ADJ_FLOPS_PER_CELL = 37  # 11 recompute + 11 adjoint + 15 gradient accumulation (FP32)


def time_pipeline(prob, subsets=3, steps=2):
    """Host-input streaming forward (the paper's workflow, Section III-A):
    pinned host arrays in, scores on the host out, H2D of the next subset
    overlapped with the current subset's compute.  Not the headline value:
    it includes the PCIe transfers."""
    from paper_2411_11547_amd import binding
    pipe = binding.Pipeline(prob, max_subset_cells=prob.total_cells // subsets + 1)
    pipe.forward()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.forward()
    sec = (time.perf_counter() - t0) / steps
    ev_ms = pipe.ms()
    nsub = pipe.num_subsets
    pipe.close()
    h2d = int(prob.read_offset[-1]) * 5 + int(prob.hap_offset[-1])
    log(f"host-input pipeline: {sec * 1e3:.2f} ms/call over {nsub} subsets, "
        f"{prob.total_cells / sec / 1e9:.1f} GCUPS")
    return {"gcups": round(prob.total_cells / sec / 1e9, 2), "ms_per_call": round(sec * 1e3, 3),
            "event_ms": round(ev_ms, 3), "subsets": nsub, "pinned": True,
            "h2d_bytes": h2d, "d2h_bytes": prob.num_pairs * 9,
            "includes": "H2D of bases and qualities, binning, FP32 sweeps, FP64 rescue, D2H of scores"}


def time_adjoint(steps, prob=None, dev=None):
    """Backward pass (checkpointed forward + reverse sweep + gradients, FP64
    for pairs outside the FP32 range), upstream gradient 1 for every pair:
    on `prob` (the mixed batch) or by default on the adjoint workload
    (10,000 pairs, 150 bp reads x 200-600 bp haplotypes)."""
    import torch
    from paper_2411_11547_amd import binding, workloads as wl
    if prob is None:
        prob = wl.config4()
    if dev is None:
        dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob, keep_checkpoints=True)
    u = torch.ones(prob.num_pairs, dtype=torch.float64, device="cuda")
    grad = torch.empty((int(prob.read_offset[-1]), 7), dtype=torch.float32, device="cuda")
    plan.backward(dev, u, grad_params=grad)
    torch.cuda.synchronize()
    ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.backward(dev, u, grad_params=grad)
        ms.append(plan.stage_ms()[3])
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    plan.close()
    cells = prob.total_cells
    kms = float(np.mean(ms))
    log(f"adjoint: {sec * 1e3:.3f} ms/step, {cells / sec / 1e9:.1f} GCUPS (stage {kms:.3f} ms)")
    return {"workload": prob.name, "pairs": prob.num_pairs, "cells": cells, "ms_per_step": round(sec * 1e3, 4),
            "gcups": round(cells / sec / 1e9, 2), "stage_ms": round(kms, 4),
            "fp32_tflops": round(ADJ_FLOPS_PER_CELL * cells / (kms * 1e-3) / 1e12, 3),
            "frac_fp32_peak": round(ADJ_FLOPS_PER_CELL * cells / (kms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)}


def single_table_file():
    """The bin table of the single persistent launch (16 lanes x K = 3..16
    rows, then 64 lanes x K = 5..16) as a tune-table file, so that both
    launch modes can run the same bins."""
    import tempfile
    lines = [f"{16 * k - 1} 16 {k}" for k in range(3, 17)] + [f"{64 * k - 1} 64 {k}" for k in range(5, 17)]
    f = tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False)
    f.write("\n".join(lines) + "\n")
    f.close()
    return f.name


def launch_ab(prob, dev, steps):
    """One persistent FP32 launch over every bin against one persistent
    launch per bin (as concurrent graph branches), on the same bin table
    (the single launch's: its kernel holds the 16-lane configurations)."""
    from paper_2411_11547_amd import binding
    path = single_table_file()
    out = {"table": "16 lanes x 3..16 rows, then 64 lanes x 5..16 rows"}
    try:
        for mode in ("bins", "single"):
            plan = binding.Plan(prob, tune_table=path, single_launch=mode == "single")
            sec, st = time_forward(plan, dev, steps, 1)
            plan.close()
            out[mode] = {"gcups": round(prob.total_cells / sec / 1e9, 2),
                         "fp32_sweep_ms": round(float(st.mean(axis=0)[1]), 4)}
            log(f"launch A/B, {mode}: {sec * 1e3:.2f} ms/step, {prob.total_cells / sec / 1e9:.1f} GCUPS")
    finally:
        os.unlink(path)
    return out


def cpu_model():
    """The host CPU's model name (as lscpu prints it), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def frac_fp32(cells, ms, flops=FLOPS_PER_CELL):
    return round(flops * cells / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)


def uniform_report(steps=10, warmup=2):
    """The uniform batch (1,000 regions x 64 reads of 150 bp x 8 haplotypes of
    300 bp, 512,000 pairs, 2.304e10 cells): binned FP32 + FP64 rescue under
    the graph, and the plain single-bin FP32 kernel, each with its FP32 sweep
    stage against the FP32 vector peak (11 flops per cell)."""
    from paper_2411_11547_amd import binding, workloads as wl
    prob = wl.config1()
    dev = binding.DeviceProblem(prob)
    cells = prob.total_cells
    rep = {"workload": prob.name, "pairs": prob.num_pairs, "cells": cells}
    for name, kw in (("binned", {}), ("plain", {"plain": True, "use_graph": False})):
        plan = binding.Plan(prob, **kw)
        sec, st = time_forward(plan, dev, steps, warmup)
        plan.close()
        ms32 = float(st.mean(axis=0)[1])
        rep[name] = {"gcups": round(cells / sec / 1e9, 2), "ms_per_step": round(sec * 1e3, 4),
                     "fp32_sweep_ms": round(ms32, 4), "frac_fp32_peak": frac_fp32(cells, ms32)}
        log(f"uniform {name}: {sec * 1e3:.3f} ms/step, {cells / sec / 1e9:.1f} GCUPS, "
            f"FP32 stage {ms32:.3f} ms ({rep[name]['frac_fp32_peak']} of peak)")
    rep["binned_vs_plain"] = round(rep["binned"]["gcups"] / rep["plain"]["gcups"], 3)
    return rep


def cpu_baseline(prob, target_cells=2.0e10, seed=0):
    import oracle
    r_idx, h_idx = prob.pair_index()
    cells = prob.pair_cells()
    order = np.random.default_rng(seed).permutation(len(cells))
    take = order[:max(1, int(np.searchsorted(np.cumsum(cells[order]), target_cells)))]
    sub_cells = int(cells[take].sum())
    t0 = time.perf_counter()
    _, used = oracle.forward(prob, pairs=np.sort(take), return_threads=True)
    dt = time.perf_counter() - t0
    return {"value": round(sub_cells / dt / 1e9, 4), "unit": "GCUPS", "cores": int(used),
            "kind": "oracle", "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
            "sample": f"{len(take)} random pairs of the same batch ({sub_cells:.3e} cells, {dt:.1f} s), "
                      "FP64 full-matrix forward, gcc -O2"}


def precision_report(steps=5):
    """Precision stress workload (50,000 pairs, 250 bp reads, 1,000-5,000 bp
    haplotypes at 5-15% divergence, 30% low-quality reads, 2% N): forward
    GCUPS, rescue fraction and per-pair |d log10 L| against the FP64 oracle,
    split by the path that produced the result."""
    import torch
    import oracle
    from paper_2411_11547_amd import binding, workloads as wl
    prob = wl.config3()
    dev = binding.DeviceProblem(prob)
    plan = binding.Plan(prob)
    sec, st = time_forward(plan, dev, steps, 2)
    out, status = plan.forward(dev)
    torch.cuda.synchronize()
    got, status = out.cpu().numpy(), status.cpu().numpy()
    plan.close()
    t0 = time.perf_counter()
    ref, used = oracle.forward(prob, return_threads=True)
    tor = time.perf_counter() - t0
    err = np.abs(got - ref)
    cells_pair = prob.pair_cells()
    resc_cells = int(cells_pair[status != 0].sum())
    ms64 = float(st.mean(axis=0)[2])
    rep = {"workload": prob.name, "pairs": prob.num_pairs, "cells": prob.total_cells,
           "gcups": round(prob.total_cells / sec / 1e9, 2), "ms_per_step": round(sec * 1e3, 3),
           "stage_ms": {"binning": round(float(st.mean(axis=0)[0]), 3),
                        "fp32_sweep": round(float(st.mean(axis=0)[1]), 3),
                        "fp64_rescue": round(ms64, 3)},
           "rescue_fraction": round(float((status != 0).mean()), 4),
           "fp64_rescue_stage": {"cells": resc_cells,
                                 "gcups": round(resc_cells / (ms64 * 1e-3) / 1e9, 2),
                                 "tflops": round(FLOPS_PER_CELL * resc_cells / (ms64 * 1e-3) / 1e12, 3),
                                 "peak": PEAK_FP64_TFLOPS,
                                 "frac_fp64_peak": round(FLOPS_PER_CELL * resc_cells / (ms64 * 1e-3) / 1e12
                                                         / PEAK_FP64_TFLOPS, 4)},
           "oracle_s": round(tor, 1), "oracle_threads": int(used),
           "log10L_range": [round(float(ref.min()), 2), round(float(ref.max()), 2)]}
    for name, code in (("fp32", 0), ("fp64", 1), ("fp64_floor", 2)):
        sel = status == code
        e = err[sel]
        rep[name] = {"pairs": int(sel.sum()), "fraction": round(float(sel.mean()), 4),
                     "max_abs_dlog10L": float(e.max()) if e.size and code != 2 else None,
                     "p99_abs_dlog10L": float(np.percentile(e, 99)) if e.size and code != 2 else None}
    log(f"precision stress: {rep['gcups']} GCUPS, rescued {rep['rescue_fraction']}, FP64 stage "
        f"{rep['fp64_rescue_stage']['frac_fp64_peak']} of the FP64 peak; FP32 max |d| "
        f"{rep['fp32']['max_abs_dlog10L']}, FP64 max |d| {rep['fp64']['max_abs_dlog10L']}")
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, help="workload index (2 = mixed-length batch)")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune-table", default=None)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-e2e", action="store_true", help="skip the host-input pipeline timing")
    ap.add_argument("--no-viterbi", action="store_true", help="skip the Viterbi timing")
    ap.add_argument("--launch", choices=["bins", "single"], default="bins",
                    help="FP32 sweep as one launch per length bin or one persistent launch")
    ap.add_argument("--no-ab", action="store_true", help="skip timing the other launch mode")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a device buffer of this many MiB (counter calibration)")
    ap.add_argument("--precision", action="store_true",
                    help="only run the precision-stress report (all pairs against the oracle)")
    ap.add_argument("--adjoint-steps", type=int, default=5)
    ap.add_argument("--no-uniform", action="store_true", help="skip the uniform-batch report")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-stress report")
    ap.add_argument("--no-adjoint-mixed", action="store_true", help="skip the adjoint on the mixed batch")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested). Each pair is independent, so sharding "
              f"would split regions across GPUs with no communication.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_11547_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    binding.load()
    if args.precision:
        print(json.dumps(precision_report()), flush=True)
        return
    log(f"generating workload {args.config}")
    prob = workload(args.config)
    cells = prob.total_cells
    log(f"{prob.name}: {prob.num_pairs} pairs, {cells:.3e} cells")
    read_len = f"{int(prob.read_lengths.min())}-{int(prob.read_lengths.max())}"
    hap_len = f"{int(prob.hap_lengths.min())}-{int(prob.hap_lengths.max())}"
    dev = binding.DeviceProblem(prob)

    plan = binding.Plan(prob, tune_table=args.tune_table, single_launch=args.launch == "single")
    sec, stages = time_forward(plan, dev, args.steps, args.warmup)
    rescued = plan.rescued()
    gcups = cells / sec / 1e9
    st_mean = stages.mean(axis=0)
    log(f"binned: {sec * 1e3:.2f} ms/step, {gcups:.1f} GCUPS, stages(ms) bin={st_mean[0]:.3f} "
        f"fp32={st_mean[1]:.3f} fp64={st_mean[2]:.3f}, rescued {rescued}")
    # the Viterbi score (max-product sweep) on the same plan and batch
    viterbi = None
    if not args.no_viterbi:
        vout = torch.empty(max(plan.num_pairs, 1), dtype=torch.float64, device="cuda")
        vstat = torch.empty(max(plan.num_pairs, 1), dtype=torch.uint8, device="cuda")
        vsec, vst = time_forward_fn(lambda: plan.viterbi(dev, out=vout, status=vstat), plan, 3, 1)
        viterbi = {"gcups": round(cells / vsec / 1e9, 2), "ms_per_step": round(vsec * 1e3, 3),
                   # 7 multiplications and 4 maxima per cell (Eq. (1)-(3) with every sum a maximum)
                   "frac_fp32_peak": frac_fp32(cells, float(vst.mean(axis=0)[1])),
                   "stage_ms": {"binning": round(float(vst.mean(axis=0)[0]), 4),
                                "fp32_sweep": round(float(vst.mean(axis=0)[1]), 4),
                                "fp64_rescue": round(float(vst.mean(axis=0)[2]), 4)},
                   "fp32_valu_per_cell": VITERBI_VALU_PER_CELL}
        log(f"viterbi: {vsec * 1e3:.2f} ms/step, {viterbi['gcups']:.1f} GCUPS")
    plan.close()

    other = None
    if not args.no_ab:
        other = launch_ab(prob, dev, max(2, args.steps // 2))

    plain = None
    if not args.no_plain:
        pplan = binding.Plan(prob, plain=True, use_graph=False)
        psec, pst = time_forward(pplan, dev, args.plain_steps, 1)
        plain = cells / psec / 1e9
        plain_ms32 = float(pst.mean(axis=0)[1])
        log(f"plain: {psec * 1e3:.2f} ms/step, {plain:.1f} GCUPS")
        pplan.close()

    t32 = st_mean[1] * 1e-3
    achieved = FLOPS_PER_CELL * cells / t32 / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": measured_traffic(prob.name),
            "kernel": "FP32 sweep stage (k_fwd32 over all length bins)",
            "kernel_ms": round(float(st_mean[1]), 4),
            "fma_slots_per_cell": FMA_SLOTS_PER_CELL,
            "fma_slot_frac": round(FMA_SLOTS_PER_CELL * cells / t32 / PEAK_FMA_LANE_OPS, 4)}

    uniform = None if args.no_uniform else uniform_report()
    precision = None if args.no_precision else precision_report()
    adj = None if args.no_adjoint else time_adjoint(args.adjoint_steps)
    adj_mixed = None if args.no_adjoint or args.no_adjoint_mixed else \
        time_adjoint(max(1, args.adjoint_steps // 2), prob, dev)
    e2e = None if args.no_e2e else time_pipeline(prob)

    cpu = None if args.no_cpu else cpu_baseline(prob)
    if cpu:
        log(f"cpu oracle: {cpu['value']} GCUPS on {cpu['cores']} threads")

    out = {"metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 (f64 rescue)", "data": "synthetic",
           "config": {"workload": prob.name, "pairs": prob.num_pairs, "cells": cells,
                      "read_len": read_len, "hap_len": hap_len, "graph": True,
                      "fp32_launch": args.launch},
           "plain_gcups": None if plain is None else round(plain, 2),
           "plain_frac_fp32_peak": None if plain is None else frac_fp32(cells, plain_ms32),
           "binned_vs_plain": None if plain is None else round(gcups / plain, 3),
           "rescued_pairs": int(rescued),
           "launch": args.launch, "other_launch": other,
           "stage_ms": {"binning": round(float(st_mean[0]), 4), "fp32_sweep": round(float(st_mean[1]), 4),
                        "fp64_rescue": round(float(st_mean[2]), 4)},
           "adjoint_gcups": None if adj is None else adj["gcups"],
           "viterbi": viterbi,
           "adjoint": adj,
           "adjoint_mixed": adj_mixed,
           "end_to_end_host_input": e2e,
           "uniform": uniform,
           "precision_stress": precision,
           "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    if args.copy_probe_mib:
        x = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        torch.cuda.synchronize()
        y = x.clone()
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written ({float(y[0]):.0f})")


if __name__ == "__main__":
    main()
