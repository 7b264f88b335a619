"""CPU checks of the C ABI: the library loads, exports every symbol that
include/ph.h declares, and rejects bad shapes before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2411_11547_amd import binding
from paper_2411_11547_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ph.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ph_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_binding_exports():
    assert set(declared_functions()) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_defaults():
    assert "gfx950" in binding.ph_version()
    o = binding.ph_plan_opts_default()
    assert o.rescue_threshold == pytest.approx(1e-28) and o.use_graph == 1 and o.plain == 0


def _plan_status(problem, **kw):
    shape, keep = binding.shape_of(problem)
    opts = binding.ph_plan_opts_default()
    for k, v in kw.items():
        setattr(opts, k, v)
    h = ctypes.c_void_p()
    st = binding.load().ph_plan_create(ctypes.byref(shape), ctypes.byref(opts), ctypes.byref(h))
    return st, binding.load().ph_last_error().decode()


def test_shape_validation_errors():
    good = wl.from_strings([(["ACGT"], ["ACGTT"])])
    # empty read
    bad = wl.from_strings([(["ACGT"], ["ACGTT"])])
    bad.read_offset[1] = 0
    bad.read_offset = np.array([0, 0], np.int64)
    st, msg = _plan_status(bad)
    assert st == -1 and "length 0" in msg
    # empty haplotype
    bad = wl.from_strings([(["ACGT"], ["ACGTT"])])
    bad.hap_offset = np.array([0, 0], np.int64)
    st, _ = _plan_status(bad)
    assert st == -1
    # read longer than the windowed sweep's limit (64 windows of 1024 rows)
    long = wl.from_strings([(["A" * 65536], ["ACGT"])])
    st, msg = _plan_status(long)
    assert st == -2 and "65536" in msg
    # batch range outside the reads
    bad = wl.from_strings([(["ACGT"], ["ACGTT"])])
    bad.batch_read_begin = np.array([0, 2], np.int32)
    st, _ = _plan_status(bad)
    assert st == -1
    # bad force_p
    st, _ = _plan_status(good, force_p=12)
    assert st == -1
    # NULL shape
    h = ctypes.c_void_p()
    assert binding.load().ph_plan_create(None, None, ctypes.byref(h)) == -1


def test_null_plan_calls():
    lib = binding.load()
    assert lib.ph_forward_batch(None, None, None, None, None, None) == -1
    assert lib.ph_backward_batch(None, None, None, None, None, None) == -1
    assert lib.ph_validate(None, None, None) == -1
    ms = (ctypes.c_float * 4)()
    assert lib.ph_plan_stage_ms(None, ms) == -1
    lib.ph_plan_destroy(None)


def test_pipeline_shape_validation_errors():
    """ph_pipeline_create rejects a bad batch range before touching the GPU."""
    bad = wl.from_strings([(["ACGT"], ["ACGTT"]), (["AC"], ["AAC"])])
    bad.batch_read_begin = np.array([0, 2, 1], np.int32)
    shape, keep = binding.shape_of(bad)
    opts = binding.ph_pipeline_opts_default()
    assert opts.plan.use_graph == 1 and opts.max_subset_cells == 0
    h = ctypes.c_void_p()
    st = binding.load().ph_pipeline_create(ctypes.byref(shape), ctypes.byref(opts), ctypes.byref(h))
    assert st == -1 and "bad read or haplotype range" in binding.load().ph_last_error().decode()
    assert not h.value


def test_struct_layout_matches_binding(tmp_path):
    """Every struct the binding mirrors has the size and field offsets that a
    C compiler gives the declarations in include/ph.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"ph_shape": binding.PhShape, "ph_problem": binding.PhProblem,
               "ph_plan_opts": binding.PhPlanOpts, "ph_pipeline_opts": binding.PhPipelineOpts}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ph.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def _noalloc_status(problem):
    shape, keep = binding.shape_of(problem)
    pb = binding.PhProblem(problem.num_batches, None, None, problem.num_reads, None, None, None, None, None,
                           None, problem.num_haps, None, None)
    st = binding.load().ph_forward_batch_noalloc(ctypes.byref(shape), ctypes.byref(pb), None, None, None, None)
    return st, binding.load().ph_last_error().decode()


def test_noalloc_rejects_sizes_beyond_its_maximum():
    """The allocation-free forward refuses, before any device work, problems
    larger than its fixed scratch: more than 65536 pairs, reads longer than
    1023 bases, more than 16384 batches."""
    many = wl.from_strings([(["ACGT"] * 257, ["ACGTT"] * 256)])  # 65792 pairs
    st, msg = _noalloc_status(many)
    assert st == -2 and "65536" in msg, msg
    long = wl.from_strings([(["A" * 1024], ["ACGT"])])
    st, msg = _noalloc_status(long)
    assert st == -2 and "1023" in msg, msg
    batches = wl.from_strings([(["A"], ["C"])] * 16385)
    st, msg = _noalloc_status(batches)
    assert st == -2 and "16384" in msg, msg
    # empty read: invalid, as for a plan
    bad = wl.from_strings([(["ACGT"], ["ACGTT"])])
    bad.read_offset = np.array([0, 0], np.int64)
    st, _ = _noalloc_status(bad)
    assert st == -1
    # counts that differ between shape and problem
    ok = wl.from_strings([(["ACGT"], ["ACGTT"])])
    shape, keep = binding.shape_of(ok)
    pb = binding.PhProblem(1, None, None, 2, None, None, None, None, None, None, 1, None, None)
    st = binding.load().ph_forward_batch_noalloc(ctypes.byref(shape), ctypes.byref(pb), None, None, None, None)
    assert st == -5


def test_tune_table_validation(tmp_path):
    """A bin table is read before any GPU call: unknown configurations,
    ranges that do not fit, and haplotype-length splits that are malformed or
    not at an edge of the binning key's buckets are rejected."""
    good = wl.from_strings([(["ACGT"], ["ACGTT"])])
    cases = [("63 16 4\n1023 64 16\n", None),
             ("63 16 4 512 64 1\n1023 64 16\n", "not compiled"),
             ("63 16 4 500 64 2\n1023 64 16\n", "bucket edge"),
             ("63 16 4 1100 64 2\n1023 64 16\n", "bucket edge"),
             ("63 16 4 1024 64\n1023 64 16\n", "bad haplotype-length split"),
             ("63 16 4 1024 32 1\n1023 64 16\n", "not compiled"),
             ("200 16 4\n1023 64 16\n", "exceeds P*K-1"),
             ("63 16 4 1152 64 2  # comment 64x4:1\n1023 64 16\n", None)]
    for text, err in cases:
        path = tmp_path / "t.txt"
        path.write_text(text)
        st, msg = _plan_status(good, tune_table_path=str(path).encode())
        if err is None:
            # a valid table: plan creation goes on to the GPU, which this host lacks
            assert "table" not in msg and "split" not in msg, (text, msg)
        else:
            assert st in (-1, -2) and err in msg, (text, st, msg)


def test_work_lists_cover_every_pair(tmp_path):
    """The FP32 work lists a binned plan builds on the host (chains of a
    batch's haplotypes per read, single pairs) cover every pair exactly once;
    plan creation checks that before its first HIP call, so on a host without
    a GPU it fails there and not on the lists.  Mixed and ragged shapes, with
    the built-in table, a table whose split sends chains to a second bin, and
    every forced group size."""
    rng = np.random.default_rng(5)
    probs = [wl.config2(regions=30), wl.config1(regions=3)]
    batches = []
    for q in range(12):
        ms = rng.integers(1, 1100, size=int(rng.integers(0, 12)))
        ns = rng.choice([1, 5, 40, 63, 64, 65, 100, 300, 700, 1500, 2100], size=int(rng.integers(0, 9)))
        batches.append(([("A" * int(m)) for m in ms], [("C" * int(n)) for n in ns]))
    probs.append(wl.from_strings(batches))
    split = tmp_path / "split.txt"
    split.write_text("223 16 14\n255 16 16 256 32 8\n1023 64 16\n")
    for prob in probs:
        for kw in (dict(), dict(tune_table_path=str(split).encode()), dict(force_p=16), dict(force_p=32),
                   dict(force_p=64)):
            st, msg = _plan_status(prob, **kw)
            assert "work lists" not in msg, (kw, msg)
            assert st == -4 or st == 0, (kw, st, msg)
