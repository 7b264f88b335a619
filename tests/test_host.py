"""CPU checks of the host-side Python around the library: the seeded workload
generators against their stated recipes and sizes, the autotuner's range
table and the committed bin table, the benchmark's one-GPU guard, and the
counter summaries that feed the benchmark's roofline traffic."""
import os
import sqlite3
import subprocess
import sys

import numpy as np

from paper_2411_11547_amd import tune
from paper_2411_11547_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _common(p):
    assert p.read_bases.max() <= 4 and p.hap_bases.max() <= 4
    assert len(p.base_qual) == len(p.read_bases) == p.read_offset[-1]
    assert len(p.hap_bases) == p.hap_offset[-1]
    assert np.all(p.read_lengths >= 1) and np.all(p.hap_lengths >= 1)


def test_config0_and_determinism():
    a, b = wl.config0(), wl.config0()
    _common(a)
    assert a.num_pairs == 32 and np.all(a.read_lengths == 100)
    for f in ("read_bases", "hap_bases", "base_qual", "ins_qual", "del_qual", "gcp_qual", "hap_offset"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.all(a.ins_qual == 45) and np.all(a.del_qual == 45) and np.all(a.gcp_qual == 10)


def test_uniform_batch_recipe():
    p = wl.config1()
    _common(p)
    assert p.num_pairs == 512_000 and p.total_cells == 512_000 * 150 * 300
    assert np.all(p.read_lengths == 150) and np.all(p.hap_lengths == 300)
    assert p.ins_qual.min() >= 40 and p.ins_qual.max() <= 45 and np.all(p.gcp_qual == 10)
    # Illumina-like base qualities: 60% Q37
    assert abs(np.mean(p.base_qual == 37) - 0.60) < 0.01


def test_mixed_batch_recipe():
    p = wl.config2()
    _common(p)
    assert p.num_pairs == 3_757_266 and p.total_cells == 222_196_841_342
    assert p.read_lengths.min() >= 50 and p.read_lengths.max() <= 250
    assert p.hap_lengths.min() >= 100 and p.hap_lengths.max() <= 2000
    haps_per_region = np.diff(p.batch_hap_begin)
    assert haps_per_region.min() >= 1 and haps_per_region.max() <= 64
    assert np.all(p.gcp_qual == 10)


def test_precision_stress_and_adjoint_recipes():
    p = wl.config3(pairs=2000)
    _common(p)
    assert p.num_pairs == 2000 and np.all(p.read_lengths == 250)
    assert p.hap_lengths.min() >= 1000 and p.hap_lengths.max() <= 5000
    q = wl.config4(pairs=500)
    _common(q)
    assert q.num_pairs == 500 and np.all(q.read_lengths == 150)
    # reference length U{200..600}; the haplotype carries up to a 5-base indel
    assert q.hap_lengths.min() >= 195 and q.hap_lengths.max() <= 605


def test_tune_ranges_cover_every_read_length():
    rs = tune.ranges()
    assert rs[0][0] == 1 and rs[-1][1] == 1023
    for (a0, a1), (b0, b1) in zip(rs, rs[1:]):
        assert b0 == a1 + 1 and a0 <= a1
    for lo, hi in rs:
        # every range ends on a P*K - 1 boundary of some compiled configuration
        assert any(p * k - 1 == hi for p, k in tune.CONFIGS) or hi % 4 == 3


def test_committed_bin_table():
    entries = []
    with open(tune.DEFAULT_TABLE) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                entries.append(tuple(int(x) for x in line.split()))
    assert entries, "empty table"
    max_m = [e[0] for e in entries]
    assert max_m == sorted(max_m) and len(set(max_m)) == len(max_m) and max_m[-1] == 1023
    for e in entries:
        assert len(e) in (3, 6), e
        m = e[0]
        for p, k in (e[1:3], e[3 + 1:6]) if len(e) == 6 else (e[1:3],):
            assert (p, k) in tune.CONFIGS, e
            assert p * k - 1 >= m, e  # the absorbing row fits
        if len(e) == 6:  # a haplotype-length split at a bucket edge of the binning key
            assert (e[3] < 1024 and e[3] % 16 == 0) or (e[3] >= 1024 and (e[3] - 1024) % 128 == 0), e
    rows = tune.read_table(tune.DEFAULT_TABLE)
    assert [r[0] for r in rows] == max_m and any(r[5] for r in rows)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _fake_counter_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real, "
                "dispatch_id integer, duration integer)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_profsum_traffic_scaling(tmp_path, capsys):
    """Counters are scaled by (probe MiB) / (what the counter reads for the
    probe copy); only forward FP32 sweep dispatches count."""
    from paper_2411_11547_amd import profsum
    sweep = "void ph::k_fwd32<16, 10, false>(ph::SweepArgs, int)"
    vit = "void ph::k_fwd32<16, 10, true>(ph::SweepArgs, int)"
    copy = "__amd_rocclr_copyBuffer"
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    # FETCH_SIZE reads half of the 1 MiB probe (512 KiB): scale 2
    _fake_counter_db(fdb, [(sweep, "FETCH_SIZE", 100.0, 1, 10), (sweep, "FETCH_SIZE", 50.0, 2, 10),
                           (vit, "FETCH_SIZE", 999.0, 3, 10), (copy, "FETCH_SIZE", 512.0, 4, 10)])
    _fake_counter_db(wdb, [(sweep, "WRITE_SIZE", 30.0, 1, 10), (copy, "WRITE_SIZE", 1024.0, 2, 10)])
    profsum.traffic(fdb, wdb, 1)
    out = capsys.readouterr().out
    line = [l for l in out.splitlines() if l.startswith("traffic_bytes_per_launch")][0]
    want = (150.0 * 2.0 + 30.0 * 1.0) * 1024.0
    assert abs(float(line.split(":")[1]) - want) <= 1e-6 * want


def test_measured_traffic_needs_matching_sources(tmp_path, monkeypatch):
    import bench
    sha = bench.forward_sources_sha256()
    assert len(sha) == 64 and int(sha, 16) >= 0
    # comments and layout do not enter the hash; code does
    assert bench._code_tokens("int a; // x\n/* y\n z */  int b;") == "int a; int b;"
    assert bench._code_tokens("int a;") != bench._code_tokens("int b;")
    prof = tmp_path / "t.txt"
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    prof.write_text(f"# comment: x\ntraffic_bytes_per_launch: 1.5e9\nworkload: w1\nforward_sources_sha256: {sha}\n")
    assert bench.measured_traffic("w1") == 1.5e9
    assert bench.measured_traffic("w2") is None
    prof.write_text("traffic_bytes_per_launch: 1.5e9\nworkload: w1\nforward_sources_sha256: 00\n")
    assert bench.measured_traffic("w1") is None


def _chain_clearing_schedule(P, ns, sep=6, chunk=None):
    """The clearing schedule of a chain tile, step by step as the FP32 sweep
    keeps it (wave-uniform bookkeeping, runs of steps in ring chunks): for
    each (lane, haplotype boundary) the step at which the lane clears."""
    cw = sep - 2
    chunk = chunk or (64 if P == 64 else 32)
    H = len(ns)
    total = (sum(ns) + sep * (H - 1) + P + 2) & ~1
    st = dict(kc=0, cpos=0, nk=0, bA=0, rs=1 << 31)
    if H > 1:
        st.update(nk=ns[0], bA=ns[0] + 2, rs=(ns[0] + 2 + cw - 1) & ~1)
    clears = {}

    def clear(step):
        assert step == st["rs"], "a clearing step fell behind the sweep"
        lo, hi = st["rs"] - st["bA"] - cw, st["rs"] - st["bA"]
        for t in range(max(lo + 1, 0), min(hi, P - 1) + 1):
            assert (t, st["kc"]) not in clears
            clears[(t, st["kc"])] = step
        if hi >= P - 1:
            st["cpos"] += st["nk"] + sep
            st["kc"] += 1
            st["nk"] = ns[st["kc"]]
            if st["kc"] < H - 1:
                st["bA"] = st["cpos"] + st["nk"] + 2
                st["rs"] = (st["bA"] + cw - 1) & ~1
            else:
                st["rs"] = 1 << 31
        else:
            st["rs"] += cw

    for s0 in range(0, total, chunk):
        cnt = min(chunk, total - s0)
        u = 0
        while True:
            stop = min(st["rs"] - s0, cnt)
            u = max(u, stop if stop > u else u)
            if u >= cnt:
                break
            clear(s0 + u)
    return clears


def test_chain_clearing_schedule():
    """Every lane of a chain tile clears its states exactly once per
    haplotype boundary, at a step where it sweeps one of the four separator
    columns from the third on (the absorbing row's sum is complete and every
    state of the real rows is zero from there), for every group size and
    haplotypes of 64 bases or more after the first (the plan's rule); and
    the schedule breaks when a later haplotype is much shorter than a
    64-lane group."""
    rng = np.random.default_rng(1)
    for P in (4, 8, 16, 32, 64):
        for _ in range(400):
            H = int(rng.integers(2, 9))
            ns = [int(rng.integers(1, 400))] + [int(rng.integers(64, 400)) for _ in range(H - 1)]
            clears = _chain_clearing_schedule(P, ns)
            assert len(clears) == P * (H - 1)
            cpos = 0
            for k in range(H - 1):
                first_sep = cpos + ns[k]
                for t in range(P):
                    pos = clears[(t, k)] - t
                    assert first_sep + 2 <= pos < first_sep + 6, (P, ns, k, t, pos)
                cpos += ns[k] + 6
    try:
        _chain_clearing_schedule(64, [300, 20, 300])
    except AssertionError:
        pass
    else:
        raise AssertionError("a 20-base haplotype inside a 64-lane chain went unnoticed")
