"""Summaries of rocprofv3 output (rocpd SQLite databases) for the profiles
kept with the repository.

    python -m paper_2411_11547_amd.profsum kernels DB
        per-kernel statistics, and the span of every forward call's FP32 sweep
        stage and of every backward call's adjoint kernels
    python -m paper_2411_11547_amd.profsum counters DB [DB ...]
        per-dispatch PMC counter values of the library's kernels and copies
    python -m paper_2411_11547_amd.profsum traffic FETCH_DB WRITE_DB COPY_MIB [KERNEL]
        HBM bytes of one forward call's FP32 sweep kernels from a FETCH_SIZE
        run and a WRITE_SIZE run of the same command, each scaled by what the
        counter reads for a device copy of COPY_MIB MiB (bench.py
        --copy-probe-mib) in the same run; with KERNEL (a name prefix such as
        k_adj32 or k_fwd64), the same scaled bytes per dispatch of every
        kernel of that name instead

Reads the databases only; runs nothing.
"""
from __future__ import annotations

import collections
import sqlite3
import sys

SWEEP = ("k_fwd32", "k_plain32", "k_long32")
ADJ = ("k_adj32", "k_adj64", "k_adj_reduce")


def _is_sweep(name):
    """A forward FP32 sweep kernel (not a Viterbi instance: those carry a
    `true` template argument)."""
    return any(k in name for k in SWEEP) and ", true>" not in name and "<true>" not in name


def _kernels(db):
    cur = sqlite3.connect(db).cursor()
    return cur.execute("select name, start, end, duration, grid_x, vgpr_count, accum_vgpr_count, "
                       "lds_size, scratch_size from kernels order by start").fetchall()


def _spans(rows, start_markers, members):
    """Span (ms) from the first to the last dispatch of `members` after each
    dispatch whose name contains one of `start_markers`."""
    spans, lo, hi = [], None, None
    for name, s, e, *_ in rows:
        if any(mk in name for mk in start_markers):
            if lo is not None:
                spans.append((hi - lo) / 1e6)
            lo = hi = None
        elif any(k in name for k in members):
            lo = s if lo is None else min(lo, s)
            hi = e if hi is None else max(hi, e)
    if lo is not None:
        spans.append((hi - lo) / 1e6)
    return spans


def kernels(db):
    rows = _kernels(db)
    stats = collections.OrderedDict()
    for name, s, e, d, gx, vg, ag, lds, scr in rows:
        st = stats.setdefault(name, [0, 0.0, gx, vg, ag, lds, scr])
        st[0] += 1
        st[1] += d
    print(f"{'kernel':<52} {'calls':>5} {'total_ms':>10} {'avg_ms':>9} {'grid':>7} {'vgpr':>5} {'agpr':>5} "
          f"{'lds':>6} {'scratch':>7}")
    for name, (c, tot, gx, vg, ag, lds, scr) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        print(f"{name[:52]:<52} {c:>5} {tot / 1e6:>10.3f} {tot / c / 1e6:>9.3f} {gx:>7} {vg:>5} {ag:>5} "
              f"{lds:>6} {scr:>7}")
    fwd = [r for r in rows if not any(k in r[0] for k in SWEEP) or _is_sweep(r[0])]
    vit = [r for r in rows if not any(k in r[0] for k in SWEEP) or not _is_sweep(r[0])]
    # a forward call starts with its binning (k_reset) or, with work lists
    # built at plan creation, with the copy of the plan's book (k_book_copy)
    first = ("k_reset", "k_book_copy")
    for title, rs, marker, members in (("FP32 sweep stage of the forward calls", fwd, first, SWEEP),
                                       ("FP32 sweep stage of the Viterbi calls", vit, first, SWEEP),
                                       ("adjoint kernels", rows, ("k_zero_i32",), ADJ)):
        sp = [x for x in _spans(rs, marker, members) if x > 0]
        if not sp:
            continue
        print()
        print(f"{title}: span per call (first dispatch start to last dispatch end), ms:")
        print("  " + " ".join(f"{x:.3f}" for x in sp))
        if len(sp) > 1:
            print(f"  mean over calls after the first: {sum(sp[1:]) / len(sp[1:]):.3f}")


def _counters(db):
    cur = sqlite3.connect(db).cursor()
    out = collections.OrderedDict()
    for name, ctr, val, disp, dur in cur.execute(
            "select kernel_name, counter_name, sum(value), dispatch_id, max(duration) from counters_collection "
            "group by dispatch_id, counter_name order by dispatch_id"):
        out.setdefault((disp, name), {})[ctr] = (val, dur)
    return out


def _interesting(name):
    return name.startswith("void ph::") or name.startswith("ph::") or "copy" in name.lower() \
        or "elementwise" in name.lower() or "fill" in name.lower()


def counters(*dbs):
    for db in dbs:
        for (disp, name), ctrs in _counters(db).items():
            if not _interesting(name):
                continue
            dur = max(d for _, d in ctrs.values()) / 1e6
            cs = " ".join(f"{k}={v:.6g}" for k, (v, _) in sorted(ctrs.items()))
            print(f"disp={disp:<5} {name[:60]:<60} dur_ms={dur:.4f} {cs}")


def _copy_and_sweep(db, counter):
    rows = _counters(db)
    sweep = 0.0
    copy = None
    for (disp, name), ctrs in rows.items():
        if counter not in ctrs:
            continue
        v = ctrs[counter][0]
        if _is_sweep(name):
            sweep += v
        elif not name.startswith(("void ph::", "ph::")) and "copy" in name.lower():
            copy = v if copy is None else max(copy, v)  # the probe is the largest copy of the run
    return sweep, copy


def traffic(fetch_db, write_db, copy_mib):
    copy_kib = float(copy_mib) * 1024.0
    f_sweep, f_copy = _copy_and_sweep(fetch_db, "FETCH_SIZE")
    w_sweep, w_copy = _copy_and_sweep(write_db, "WRITE_SIZE")
    ff = copy_kib / f_copy if f_copy else float("nan")
    fw = copy_kib / w_copy if w_copy else float("nan")
    fetch_b = f_sweep * ff * 1024.0
    write_b = w_sweep * fw * 1024.0
    print(f"copy probe {copy_mib} MiB: FETCH_SIZE read {f_copy:.6g} KiB (scale {ff:.4f}), "
          f"WRITE_SIZE read {w_copy:.6g} KiB (scale {fw:.4f})")
    print(f"FP32 sweep kernels of the call: FETCH_SIZE {f_sweep:.6g} KiB, WRITE_SIZE {w_sweep:.6g} KiB")
    print(f"HBM traffic per FP32 sweep stage (scaled): fetch {fetch_b:.6g} B + write {write_b:.6g} B "
          f"= {fetch_b + write_b:.6g} B")
    print(f"traffic_bytes_per_launch: {fetch_b + write_b:.6g}")


def traffic_kernel(fetch_db, write_db, copy_mib, prefix):
    copy_kib = float(copy_mib) * 1024.0
    out = {}
    for db, counter in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        copy = None
        per = collections.OrderedDict()
        for (disp, name), ctrs in _counters(db).items():
            if counter not in ctrs:
                continue
            v, dur = ctrs[counter]
            if prefix in name:
                e = per.setdefault(name, [0, 0.0, 0.0])
                e[0] += 1
                e[1] += v
                e[2] += dur
            elif not name.startswith(("void ph::", "ph::")) and "copy" in name.lower():
                copy = v if copy is None else max(copy, v)
        scale = copy_kib / copy if copy else float("nan")
        print(f"copy probe {copy_mib} MiB: {counter} read {copy:.6g} KiB (scale {scale:.4f})")
        for name, (n, v, dur) in per.items():
            out.setdefault(name, {})[counter] = (n, v * scale * 1024.0 / n, dur / n / 1e6)
    for name, d in out.items():
        f = d.get("FETCH_SIZE", (0, float("nan"), 0))
        w = d.get("WRITE_SIZE", (0, float("nan"), 0))
        print(f"{name}: {f[0]} dispatches; per dispatch fetch {f[1]:.6g} B + write {w[1]:.6g} B "
              f"= {f[1] + w[1]:.6g} B, mean duration {f[2]:.4f} / {w[2]:.4f} ms")


def main(argv):
    if len(argv) >= 2 and argv[0] == "kernels":
        kernels(argv[1])
    elif len(argv) >= 2 and argv[0] == "counters":
        counters(*argv[1:])
    elif len(argv) == 4 and argv[0] == "traffic":
        traffic(argv[1], argv[2], argv[3])
    elif len(argv) == 5 and argv[0] == "traffic":
        traffic_kernel(argv[1], argv[2], argv[3], argv[4])
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
