"""FP64 CPU oracle for the Pair-HMM forward algorithm and its adjoint.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  It shares no code with the HIP path.

`pairhmm_oracle.c` holds the arithmetic (plain full-matrix FP64 DP, Section
II-A Eq. (1)-(4) and the initialisation and result formulas that follow them);
this module builds it with gcc and marshals arguments through ctypes.
`bruteforce.py` enumerates alignment paths one by one for tiny pairs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pairhmm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
NCH = 7
CHANNELS = ("alpha", "beta", "delta", "eps", "zeta", "lam_match", "lam_mismatch")
EXT_CHANNELS = ("alpha", "beta", "delta", "eps_I", "eps_D", "zeta", "lam_match", "lam_mismatch")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no hand-written SIMD)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.oracle_forward.restype = ctypes.c_double
        lib.oracle_forward.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int]
        lib.oracle_forward_full.restype = ctypes.c_int
        lib.oracle_forward_full.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P]
        lib.oracle_backward.restype = ctypes.c_int
        lib.oracle_backward.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P]
        lib.oracle_params_from_phred.restype = None
        lib.oracle_params_from_phred.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.oracle_forward_pairs.restype = ctypes.c_int
        lib.oracle_forward_pairs.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, P,
                                             ctypes.c_int, ctypes.c_int, P]
        lib.oracle_viterbi.restype = ctypes.c_double
        lib.oracle_viterbi.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int]
        lib.oracle_viterbi_pairs.restype = ctypes.c_int
        lib.oracle_viterbi_pairs.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, P,
                                             ctypes.c_int, ctypes.c_int, P]
        lib.oracle_backward_pairs.restype = ctypes.c_int
        lib.oracle_backward_pairs.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, P,
                                              ctypes.c_int, ctypes.c_int, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# --- single pair -------------------------------------------------------------
def params_from_phred(bq, iq, dq, gq) -> np.ndarray:
    """[m, 7] FP64 {alpha, beta, delta, eps, zeta, lam_match, lam_mismatch}."""
    bq, iq, dq, gq = map(_u8, (bq, iq, dq, gq))
    m = len(bq)
    out = np.empty((m, NCH), np.float64)
    _load().oracle_params_from_phred(m, _p(bq), _p(iq), _p(dq), _p(gq), _p(out))
    return out


def forward_pair(read, hap, params, rescale=True, literal_n=False) -> float:
    """log10 L of one pair from per-position parameters [m, 7]."""
    read, hap, params = _u8(read), _u8(hap), _f64(params)
    assert params.shape == (len(read), NCH)
    return _load().oracle_forward(len(read), len(hap), _p(read), _p(hap), _p(params),
                                  int(rescale), int(literal_n))


def viterbi_pair(read, hap, params, rescale=True, literal_n=False) -> float:
    """log10 of the most probable alignment path's probability (max-product
    form of Eq. (1)-(3), result max_j of M(m,j), I(m,j))."""
    read, hap, params = _u8(read), _u8(hap), _f64(params)
    assert params.shape == (len(read), NCH)
    return _load().oracle_viterbi(len(read), len(hap), _p(read), _p(hap), _p(params),
                                  int(rescale), int(literal_n))


def forward_matrices(read, hap, params, literal_n=False):
    """Unscaled M, I, D, each (m+1) x (n+1)."""
    read, hap, params = _u8(read), _u8(hap), _f64(params)
    m, n = len(read), len(hap)
    M = np.empty((m + 1, n + 1)); I = np.empty_like(M); D = np.empty_like(M)
    rc = _load().oracle_forward_full(m, n, _p(read), _p(hap), _p(params), int(literal_n),
                                     _p(M), _p(I), _p(D))
    if rc:
        raise ValueError("oracle_forward_full failed")
    return M, I, D


def backward_pair(read, hap, params, literal_n=False):
    """(grad_ext [m, 8], log10 L forward, log10 L from the backward total)."""
    read, hap, params = _u8(read), _u8(hap), _f64(params)
    m, n = len(read), len(hap)
    g = np.empty((m, 8))
    lf = ctypes.c_double(); lb = ctypes.c_double()
    rc = _load().oracle_backward(m, n, _p(read), _p(hap), _p(params), int(literal_n), _p(g),
                                 ctypes.byref(lf), ctypes.byref(lb))
    if rc:
        raise ValueError("oracle_backward failed")
    return g, lf.value, lb.value


def ext_to_7(g_ext: np.ndarray) -> np.ndarray:
    """Fold the eps_I / eps_D split back into the tied eps channel."""
    g = np.empty(g_ext.shape[:-1] + (NCH,))
    g[..., 0:3] = g_ext[..., 0:3]
    g[..., 3] = g_ext[..., 3] + g_ext[..., 4]
    g[..., 4:7] = g_ext[..., 5:8]
    return g


# --- batches -----------------------------------------------------------------
def forward(problem, log10_params=None, pairs=None, literal_n=False, threads=None,
            return_threads=False):
    """log10 L for every pair of `problem` in output order (or for the output
    indices in `pairs`).  log10_params: optional float32 [sum m, 7]."""
    r, h = problem.pair_index()
    if pairs is not None:
        pairs = np.asarray(pairs, dtype=np.int64)
        r, h = r[pairs], h[pairs]
    r = np.ascontiguousarray(r, np.int32); h = np.ascontiguousarray(h, np.int32)
    out = np.empty(len(r), np.float64)
    lp = None if log10_params is None else np.ascontiguousarray(log10_params, np.float32)
    thr = threads or default_threads()
    used = _load().oracle_forward_pairs(len(r), _p(r), _p(h), _p(problem.read_offset),
                                        _p(problem.read_bases), _p(problem.base_qual),
                                        _p(problem.ins_qual), _p(problem.del_qual),
                                        _p(problem.gcp_qual), _p(problem.hap_offset),
                                        _p(problem.hap_bases), _p(lp), int(literal_n), thr,
                                        _p(out))
    return (out, used) if return_threads else out


def viterbi(problem, log10_params=None, pairs=None, literal_n=False, threads=None):
    """log10 of the best path's probability for every pair (or the output
    indices in `pairs`), in output order."""
    r, h = problem.pair_index()
    if pairs is not None:
        pairs = np.asarray(pairs, dtype=np.int64)
        r, h = r[pairs], h[pairs]
    r = np.ascontiguousarray(r, np.int32); h = np.ascontiguousarray(h, np.int32)
    out = np.empty(len(r), np.float64)
    lp = None if log10_params is None else np.ascontiguousarray(log10_params, np.float32)
    _load().oracle_viterbi_pairs(len(r), _p(r), _p(h), _p(problem.read_offset),
                                 _p(problem.read_bases), _p(problem.base_qual),
                                 _p(problem.ins_qual), _p(problem.del_qual),
                                 _p(problem.gcp_qual), _p(problem.hap_offset),
                                 _p(problem.hap_bases), _p(lp), int(literal_n),
                                 threads or default_threads(), _p(out))
    return out


def backward(problem, log10_params=None, pairs=None, literal_n=False, threads=None):
    """Per-pair gradients d log10 L / d log10 theta.

    Returns (log10L [P], grad [sum over pairs of m, 7], row_offset [P+1],
    grad_ext [.., 8]); the rows of pair k are row_offset[k]:row_offset[k+1]."""
    r, h = problem.pair_index()
    if pairs is not None:
        pairs = np.asarray(pairs, dtype=np.int64)
        r, h = r[pairs], h[pairs]
    r = np.ascontiguousarray(r, np.int32); h = np.ascontiguousarray(h, np.int32)
    m = problem.read_lengths[r].astype(np.int64)
    off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    g = np.zeros((int(off[-1]), 8))
    out = np.empty(len(r))
    lp = None if log10_params is None else np.ascontiguousarray(log10_params, np.float32)
    _load().oracle_backward_pairs(len(r), _p(r), _p(h), _p(problem.read_offset),
                                  _p(problem.read_bases), _p(problem.base_qual),
                                  _p(problem.ins_qual), _p(problem.del_qual),
                                  _p(problem.gcp_qual), _p(problem.hap_offset),
                                  _p(problem.hap_bases), _p(lp), int(literal_n),
                                  threads or default_threads(), _p(off[:-1].copy()), _p(g),
                                  _p(out))
    return out, ext_to_7(g), off, g
