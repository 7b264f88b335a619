"""ctypes binding of libpairhmm (include/ph.h): argument marshalling only.

Every step of the Pair-HMM path runs in the HIP kernels behind the C ABI;
this module converts arrays to device tensors (torch is used for device
memory and streams only), fills the C structs and calls the entry points of
the same names.  There is no CPU fallback: if the library is missing or the
GPU is unavailable, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the library this process loads: libpairhmm.so next to this file, unless
# PAIRHMM_LIBRARY names another build of it (e.g. libpairhmm_ftz.so)
LIB_PATH = os.environ.get("PAIRHMM_LIBRARY") or os.path.join(HERE, "libpairhmm.so")
# bin table measured by tune.py on MI355X; "builtin" selects the library's own
TUNED_TABLE = os.path.join(HERE, "tune_gfx950.txt")

PH_OK = 0
STATUS_NAMES = {0: "PH_OK", -1: "PH_ERR_INVALID", -2: "PH_ERR_UNSUPPORTED", -3: "PH_ERR_NOMEM",
                -4: "PH_ERR_HIP", -5: "PH_ERR_PLAN_MISMATCH", -6: "PH_ERR_STATE"}
PAIR_FP32, PAIR_FP64, PAIR_FP64_FLOOR, PAIR_FP32_UNRESCUED = 0, 1, 2, 3

EXPORTS = ("ph_plan_opts_default", "ph_plan_create", "ph_plan_info", "ph_forward_batch", "ph_viterbi_batch",
           "ph_forward_batch_noalloc",
           "ph_backward_batch", "ph_validate", "ph_plan_stage_ms", "ph_plan_rescued",
           "ph_plan_destroy", "ph_last_error", "ph_version",
           "ph_pipeline_opts_default", "ph_pipeline_create", "ph_pipeline_info", "ph_pipeline_forward",
           "ph_pipeline_ms", "ph_pipeline_destroy", "ph_host_alloc", "ph_host_free")

_p = ctypes.c_void_p


class PhShape(ctypes.Structure):
    _fields_ = [("num_batches", ctypes.c_int32), ("batch_read_begin", _p), ("batch_hap_begin", _p),
                ("num_reads", ctypes.c_int32), ("read_offset", _p),
                ("num_haps", ctypes.c_int32), ("hap_offset", _p)]


class PhProblem(ctypes.Structure):
    _fields_ = [("num_batches", ctypes.c_int32), ("batch_read_begin", _p), ("batch_hap_begin", _p),
                ("num_reads", ctypes.c_int32), ("read_offset", _p), ("read_bases", _p),
                ("base_qual", _p), ("ins_qual", _p), ("del_qual", _p), ("gcp_qual", _p),
                ("num_haps", ctypes.c_int32), ("hap_offset", _p), ("hap_bases", _p)]


class PhPlanOpts(ctypes.Structure):
    _fields_ = [("rescue_threshold", ctypes.c_double), ("use_graph", ctypes.c_int),
                ("plain", ctypes.c_int), ("force_p", ctypes.c_int),
                ("keep_checkpoints", ctypes.c_int), ("tune_table_path", ctypes.c_char_p),
                ("single_launch", ctypes.c_int)]


class PhPipelineOpts(ctypes.Structure):
    _fields_ = [("max_subset_cells", ctypes.c_int64), ("buffer_sets", ctypes.c_int32), ("plan", PhPlanOpts)]


class PHError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpairhmm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2411_11547_amd/build.py")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.ph_plan_opts_default.argtypes = [ctypes.POINTER(PhPlanOpts)]
    lib.ph_plan_opts_default.restype = None
    lib.ph_plan_create.argtypes = [ctypes.POINTER(PhShape), ctypes.POINTER(PhPlanOpts), ctypes.POINTER(P)]
    lib.ph_plan_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.ph_forward_batch.argtypes = [P, ctypes.POINTER(PhProblem), P, P, P, P]
    lib.ph_viterbi_batch.argtypes = [P, ctypes.POINTER(PhProblem), P, P, P, P]
    lib.ph_forward_batch_noalloc.argtypes = [ctypes.POINTER(PhShape), ctypes.POINTER(PhProblem), P, P, P, P]
    lib.ph_backward_batch.argtypes = [P, ctypes.POINTER(PhProblem), P, P, P, P]
    lib.ph_validate.argtypes = [P, ctypes.POINTER(PhProblem), P]
    lib.ph_plan_stage_ms.argtypes = [P, ctypes.POINTER(ctypes.c_float)]
    lib.ph_plan_rescued.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.ph_plan_destroy.argtypes = [P]
    lib.ph_plan_destroy.restype = None
    lib.ph_last_error.restype = ctypes.c_char_p
    lib.ph_last_error.argtypes = []
    lib.ph_version.restype = ctypes.c_char_p
    lib.ph_version.argtypes = []
    lib.ph_pipeline_opts_default.argtypes = [ctypes.POINTER(PhPipelineOpts)]
    lib.ph_pipeline_opts_default.restype = None
    lib.ph_pipeline_create.argtypes = [ctypes.POINTER(PhShape), ctypes.POINTER(PhPipelineOpts),
                                       ctypes.POINTER(P)]
    lib.ph_pipeline_info.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.ph_pipeline_forward.argtypes = [P, ctypes.POINTER(PhProblem), P, P]
    lib.ph_pipeline_ms.argtypes = [P, ctypes.POINTER(ctypes.c_float)]
    lib.ph_pipeline_destroy.argtypes = [P]
    lib.ph_pipeline_destroy.restype = None
    lib.ph_host_alloc.argtypes = [ctypes.c_size_t]
    lib.ph_host_alloc.restype = P
    lib.ph_host_free.argtypes = [P]
    lib.ph_host_free.restype = None
    for name in ("ph_plan_create", "ph_plan_info", "ph_forward_batch", "ph_viterbi_batch", "ph_backward_batch",
                 "ph_forward_batch_noalloc",
                 "ph_validate", "ph_plan_stage_ms", "ph_plan_rescued", "ph_pipeline_create",
                 "ph_pipeline_info", "ph_pipeline_forward", "ph_pipeline_ms"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != PH_OK:
        raise PHError(status, load().ph_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _torch():
    import torch  # device memory and streams only
    return torch


def current_stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class DeviceProblem:
    """The arrays of a `workloads.Problem` as device tensors plus the C struct."""

    FIELDS = ("batch_read_begin", "batch_hap_begin", "read_offset", "read_bases", "base_qual",
              "ins_qual", "del_qual", "gcp_qual", "hap_offset", "hap_bases")

    def __init__(self, problem, device="cuda"):
        torch = _torch()
        self.problem = problem
        self.t = {}
        for f in self.FIELDS:
            arr = np.ascontiguousarray(getattr(problem, f))
            if arr.size == 0:
                arr = np.zeros(1, dtype=arr.dtype)  # keep a valid device pointer
            self.t[f] = torch.from_numpy(arr).to(device)
        self.c = PhProblem(problem.num_batches, *[self._ptr(f) for f in ("batch_read_begin", "batch_hap_begin")],
                           problem.num_reads, *[self._ptr(f) for f in ("read_offset", "read_bases", "base_qual",
                                                                       "ins_qual", "del_qual", "gcp_qual")],
                           problem.num_haps, self._ptr("hap_offset"), self._ptr("hap_bases"))

    def _ptr(self, f):
        return ctypes.c_void_p(self.t[f].data_ptr())


def shape_of(problem):
    """PhShape over host arrays of a workloads.Problem (kept alive by the caller)."""
    keep = [np.ascontiguousarray(problem.batch_read_begin, np.int32),
            np.ascontiguousarray(problem.batch_hap_begin, np.int32),
            np.ascontiguousarray(problem.read_offset, np.int64),
            np.ascontiguousarray(problem.hap_offset, np.int64)]
    s = PhShape(problem.num_batches, _np_ptr(keep[0]), _np_ptr(keep[1]), problem.num_reads,
                _np_ptr(keep[2]), problem.num_haps, _np_ptr(keep[3]))
    return s, keep


# --- C ABI entry points (same names) -----------------------------------------
def ph_plan_opts_default() -> PhPlanOpts:
    o = PhPlanOpts()
    load().ph_plan_opts_default(ctypes.byref(o))
    return o


def ph_plan_create(shape: PhShape, opts: PhPlanOpts) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().ph_plan_create(ctypes.byref(shape), ctypes.byref(opts), ctypes.byref(h)))
    return h


def ph_plan_info(plan):
    P, C = ctypes.c_int64(), ctypes.c_int64()
    M, Nn = ctypes.c_int32(), ctypes.c_int32()
    _check(load().ph_plan_info(plan, ctypes.byref(P), ctypes.byref(C), ctypes.byref(M), ctypes.byref(Nn)))
    return P.value, C.value, M.value, Nn.value


def ph_forward_batch(plan, problem: PhProblem, log10_params, out_log10L, out_status, stream):
    _check(load().ph_forward_batch(plan, ctypes.byref(problem), log10_params, out_log10L, out_status, stream))


def ph_viterbi_batch(plan, problem: PhProblem, log10_params, out_log10V, out_status, stream):
    _check(load().ph_viterbi_batch(plan, ctypes.byref(problem), log10_params, out_log10V, out_status, stream))


def ph_forward_batch_noalloc(shape: PhShape, problem: PhProblem, log10_params, out_log10L, out_status, stream):
    _check(load().ph_forward_batch_noalloc(ctypes.byref(shape), ctypes.byref(problem), log10_params, out_log10L,
                                           out_status, stream))


def forward_noalloc(problem, dev, log10_params=None, out=None, status=None, stream=None):
    """ph_forward_batch_noalloc on a `workloads.Problem` and its DeviceProblem:
    (log10 L [P] float64, status [P] uint8) as device tensors."""
    torch = _torch()
    shape, keep = shape_of(problem)  # host shape arrays, read during the call
    P = int(problem.num_pairs)
    if out is None:
        out = torch.empty(max(P, 1), dtype=torch.float64, device="cuda")
    if status is None:
        status = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
    lp = None if log10_params is None else ctypes.c_void_p(log10_params.data_ptr())
    ph_forward_batch_noalloc(shape, dev.c, lp, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                             stream or current_stream())
    return out[:P], status[:P]


def ph_backward_batch(plan, problem: PhProblem, log10_params, grad_log10L, grad_params, stream):
    _check(load().ph_backward_batch(plan, ctypes.byref(problem), log10_params, grad_log10L, grad_params, stream))


def ph_validate(plan, problem: PhProblem, stream):
    _check(load().ph_validate(plan, ctypes.byref(problem), stream))


def ph_plan_stage_ms(plan):
    ms = (ctypes.c_float * 4)()
    _check(load().ph_plan_stage_ms(plan, ms))
    return list(ms)


def ph_plan_rescued(plan) -> int:
    c = ctypes.c_int64()
    _check(load().ph_plan_rescued(plan, ctypes.byref(c)))
    return c.value


def ph_plan_destroy(plan):
    load().ph_plan_destroy(plan)


def ph_version() -> str:
    return load().ph_version().decode()


def ph_pipeline_opts_default() -> PhPipelineOpts:
    o = PhPipelineOpts()
    load().ph_pipeline_opts_default(ctypes.byref(o))
    return o


def ph_pipeline_create(shape: PhShape, opts: PhPipelineOpts) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().ph_pipeline_create(ctypes.byref(shape), ctypes.byref(opts), ctypes.byref(h)))
    return h


def ph_pipeline_info(pipe):
    n, P, C = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().ph_pipeline_info(pipe, ctypes.byref(n), ctypes.byref(P), ctypes.byref(C)))
    return n.value, P.value, C.value


def ph_pipeline_forward(pipe, host_problem: PhProblem, out_log10L, out_status):
    _check(load().ph_pipeline_forward(pipe, ctypes.byref(host_problem), out_log10L, out_status))


def ph_pipeline_ms(pipe) -> float:
    ms = ctypes.c_float()
    _check(load().ph_pipeline_ms(pipe, ctypes.byref(ms)))
    return ms.value


def ph_pipeline_destroy(pipe):
    load().ph_pipeline_destroy(pipe)


def ph_host_alloc(nbytes: int) -> int:
    p = load().ph_host_alloc(max(int(nbytes), 1))
    if not p:
        raise PHError(-3, "ph_host_alloc failed")
    return p


def ph_host_free(ptr):
    load().ph_host_free(ptr)


class PinnedArray:
    """A numpy view of pinned host memory from ph_host_alloc."""

    def __init__(self, arr):
        arr = np.ascontiguousarray(arr)
        self.ptr = ph_host_alloc(arr.nbytes)
        buf = (ctypes.c_uint8 * max(arr.nbytes, 1)).from_address(self.ptr)
        self.a = np.frombuffer(buf, dtype=arr.dtype, count=arr.size).reshape(arr.shape)
        self.a[...] = arr

    def close(self):
        if self.ptr:
            self.a = None
            ph_host_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- convenience wrapper --------------------------------------------------------
class Plan:
    """A plan for one problem shape, with device output buffers."""

    def __init__(self, problem, rescue_threshold=None, use_graph=True, plain=False, force_p=0,
                 keep_checkpoints=False, tune_table=None, single_launch=False):
        opts = ph_plan_opts_default()
        if rescue_threshold is not None:
            opts.rescue_threshold = float(rescue_threshold)
        opts.use_graph = int(bool(use_graph))
        opts.plain = int(bool(plain))
        opts.force_p = int(force_p)
        opts.keep_checkpoints = int(bool(keep_checkpoints))
        opts.single_launch = int(bool(single_launch))
        # the tuned table by default; the single persistent launch takes only
        # 16-lane bins, so it gets the library's built-in table for it unless
        # a table is given
        if tune_table is None and not force_p and not single_launch and os.path.exists(TUNED_TABLE):
            tune_table = TUNED_TABLE
        if tune_table == "builtin":
            tune_table = None
        self._tune = tune_table.encode() if tune_table else None
        opts.tune_table_path = self._tune
        shape, self._keep = shape_of(problem)
        self.problem_bases = int(problem.read_offset[-1])
        self.handle = ph_plan_create(shape, opts)
        self.num_pairs, self.num_cells, self.max_read_len, self.max_hap_len = ph_plan_info(self.handle)

    def forward(self, dev: DeviceProblem, log10_params=None, out=None, status=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(max(self.num_pairs, 1), dtype=torch.float64, device="cuda")
        if status is None:
            status = torch.empty(max(self.num_pairs, 1), dtype=torch.uint8, device="cuda")
        lp = None if log10_params is None else ctypes.c_void_p(log10_params.data_ptr())
        ph_forward_batch(self.handle, dev.c, lp, ctypes.c_void_p(out.data_ptr()),
                         ctypes.c_void_p(status.data_ptr()), stream or current_stream())
        return out[:self.num_pairs], status[:self.num_pairs]

    def viterbi(self, dev: DeviceProblem, log10_params=None, out=None, status=None, stream=None):
        """log10 of each pair's best-path probability (ph_viterbi_batch)."""
        torch = _torch()
        if out is None:
            out = torch.empty(max(self.num_pairs, 1), dtype=torch.float64, device="cuda")
        if status is None:
            status = torch.empty(max(self.num_pairs, 1), dtype=torch.uint8, device="cuda")
        lp = None if log10_params is None else ctypes.c_void_p(log10_params.data_ptr())
        ph_viterbi_batch(self.handle, dev.c, lp, ctypes.c_void_p(out.data_ptr()),
                         ctypes.c_void_p(status.data_ptr()), stream or current_stream())
        return out[:self.num_pairs], status[:self.num_pairs]

    def backward(self, dev: DeviceProblem, grad_log10L, log10_params=None, grad_params=None, stream=None):
        """Gradient of sum_p grad_log10L[p] * log10 L_p w.r.t. the log10
        parameters of every read base: float32 [sum m, 7]."""
        torch = _torch()
        nb = int(self.problem_bases)
        if grad_params is None:
            grad_params = torch.empty((max(nb, 1), 7), dtype=torch.float32, device="cuda")
        g = grad_log10L.contiguous()
        assert g.dtype == torch.float64 and g.numel() >= self.num_pairs
        lp = None if log10_params is None else ctypes.c_void_p(log10_params.data_ptr())
        ph_backward_batch(self.handle, dev.c, lp, ctypes.c_void_p(g.data_ptr()),
                          ctypes.c_void_p(grad_params.data_ptr()), stream or current_stream())
        return grad_params[:nb]

    def validate(self, dev: DeviceProblem, stream=None):
        ph_validate(self.handle, dev.c, stream or current_stream())

    def stage_ms(self):
        return ph_plan_stage_ms(self.handle)

    def rescued(self) -> int:
        return ph_plan_rescued(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            ph_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pipeline:
    """Streaming forward over a host-resident problem (ph_pipeline_*): the
    problem's arrays are copied once into pinned host memory here, the calls
    then move them subset by subset."""

    DATA = ("read_bases", "base_qual", "ins_qual", "del_qual", "gcp_qual", "hap_bases")

    def __init__(self, problem, max_subset_cells=0, pinned=True, tune_table=None, buffer_sets=0, **plan_kw):
        opts = ph_pipeline_opts_default()
        opts.max_subset_cells = int(max_subset_cells)
        opts.buffer_sets = int(buffer_sets)
        for k, v in plan_kw.items():
            setattr(opts.plan, k, v)
        # the same bin table as Plan, so that every pair gets the same lane
        # count and hence the same rounding as in a resident plan
        if tune_table is None and not plan_kw.get("force_p") and os.path.exists(TUNED_TABLE):
            tune_table = TUNED_TABLE
        if tune_table == "builtin":
            tune_table = None
        self._tune = tune_table.encode() if tune_table else None
        opts.plan.tune_table_path = self._tune
        shape, self._keep = shape_of(problem)
        self.handle = ph_pipeline_create(shape, opts)
        self.num_subsets, self.num_pairs, self.num_cells = ph_pipeline_info(self.handle)
        self._host = {}
        for f in self.DATA:
            arr = np.ascontiguousarray(getattr(problem, f))
            self._host[f] = PinnedArray(arr) if pinned else arr
        self.out = PinnedArray(np.zeros(max(self.num_pairs, 1))) if pinned else np.zeros(max(self.num_pairs, 1))
        self.status = PinnedArray(np.zeros(max(self.num_pairs, 1), np.uint8)) if pinned else \
            np.zeros(max(self.num_pairs, 1), np.uint8)
        k = self._keep
        hp = lambda f: ctypes.c_void_p((self._host[f].a if pinned else self._host[f]).ctypes.data)
        self.c = PhProblem(problem.num_batches, _np_ptr(k[0]), _np_ptr(k[1]), problem.num_reads, _np_ptr(k[2]),
                           hp("read_bases"), hp("base_qual"), hp("ins_qual"), hp("del_qual"), hp("gcp_qual"),
                           problem.num_haps, _np_ptr(k[3]), hp("hap_bases"))
        self.pinned = pinned

    def _arr(self, x):
        return x.a if self.pinned else x

    def forward(self):
        """Scores (float64) and statuses (uint8) of every pair, host arrays."""
        out, st = self._arr(self.out), self._arr(self.status)
        ph_pipeline_forward(self.handle, self.c, ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(st.ctypes.data))
        return out[:self.num_pairs].copy(), st[:self.num_pairs].copy()

    def ms(self) -> float:
        return ph_pipeline_ms(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            ph_pipeline_destroy(self.handle)
            self.handle = None
        if getattr(self, "pinned", False):
            for v in list(self._host.values()) + [self.out, self.status]:
                v.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
