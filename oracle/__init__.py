"""FP64 CPU oracle for the tiled-composite SpMV path.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  The GPU library never imports, links or calls it, and it never
imports the library.

  oracle.c        plain FP64 CSR SpMV / SpMM and the PageRank, HITS and RWR
                  power iterations (ctypes, built here with gcc)
  ref_format.py   reference builder of the tiled composite format (numpy)
  autotune.py     Algorithms 1-3 and the performance model (Eq. 1-5)
  rwr_grad.py     RWR with learned, column-normalised edge weights and the
                  gradient of a loss on its iterate (FP64 adjoint pass)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so: plain C, -O3 (portable x86-64), OpenMP, no fast-math."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fno-fast-math", "-fopenmp",
                               "-ffp-contract=off", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        lib.or_spmv_f32x.argtypes = [i64, vp, vp, vp, vp, vp]
        lib.or_spmv_f64x.argtypes = [i64, vp, vp, vp, vp, vp]
        lib.or_absmv_f32x.argtypes = [i64, vp, vp, vp, vp, vp]
        lib.or_spmv_rows_f32x.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
        lib.or_spmm_f32x.argtypes = [i64, vp, vp, vp, vp, i64, vp]
        lib.or_pagerank.argtypes = [i64, vp, vp, vp, dbl, dbl, i64, vp, vp]
        lib.or_pagerank.restype = i64
        lib.or_hits.argtypes = [i64, vp, vp, vp, dbl, i64, vp, vp]
        lib.or_hits.restype = i64
        lib.or_rwr.argtypes = [i64, vp, vp, vp, vp, i64, dbl, dbl, i64, vp, vp]
        lib.or_rwr.restype = i64
        lib.or_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(csr):
    n_rows, n_cols, rp, col, val = csr
    return (int(n_rows), int(n_cols), np.ascontiguousarray(rp, np.int64),
            np.ascontiguousarray(col, np.int32), np.ascontiguousarray(val, np.float32))


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    lib = _load()
    lib.or_set_threads.argtypes = [ctypes.c_int]
    lib.or_set_threads.restype = None
    lib.or_set_threads(int(n))


def spmv(csr, x) -> np.ndarray:
    """y = A x in FP64 (x upcast from FP32 if it is FP32)."""
    n_rows, n_cols, rp, col, val = _csr(csr)
    y = np.empty(n_rows, np.float64)
    if np.asarray(x).dtype == np.float64:
        x = np.ascontiguousarray(x, np.float64)
        _load().or_spmv_f64x(n_rows, _p(rp), _p(col), _p(val), _p(x), _p(y))
    else:
        x = np.ascontiguousarray(x, np.float32)
        _load().or_spmv_f32x(n_rows, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def absmv(csr, x) -> np.ndarray:
    """(|A| |x|)_i, the scale of the per-entry error bound."""
    n_rows, n_cols, rp, col, val = _csr(csr)
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty(n_rows, np.float64)
    _load().or_absmv_f32x(n_rows, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def spmv_rows(csr, x, rows):
    """Selected rows of A x and of |A||x| (sampled checks at full size)."""
    n_rows, n_cols, rp, col, val = _csr(csr)
    rows = np.ascontiguousarray(rows, np.int64)
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty(len(rows), np.float64)
    a = np.empty(len(rows), np.float64)
    _load().or_spmv_rows_f32x(len(rows), _p(rows), _p(rp), _p(col), _p(val), _p(x), _p(y), _p(a))
    return y, a


def spmm(csr, X) -> np.ndarray:
    """Y = A X, X row-major n_cols x k FP32."""
    n_rows, n_cols, rp, col, val = _csr(csr)
    X = np.ascontiguousarray(X, np.float32)
    k = X.shape[1]
    Y = np.empty((n_rows, k), np.float64)
    _load().or_spmm_f32x(n_rows, _p(rp), _p(col), _p(val), _p(X), k, _p(Y))
    return Y


def pagerank(csr, c=0.85, tol=0.0, max_iter=50):
    """PageRank (Eq. 6, dangling mass spread uniformly) -> (p, iterations, residuals)."""
    n_rows, n_cols, rp, col, val = _csr(csr)
    p = np.empty(n_rows, np.float64)
    res = np.zeros(max(max_iter, 1), np.float64)
    it = _load().or_pagerank(n_rows, _p(rp), _p(col), _p(val), c, tol, max_iter, _p(p), _p(res))
    return p, int(it), res[:it]


def hits(csr, tol=0.0, max_iter=50):
    """HITS on [[0, A^T], [A, 0]] -> (x = [a; h], iterations, residuals)."""
    n2, _, rp, col, val = _csr(csr)
    x = np.empty(n2, np.float64)
    res = np.zeros(max(max_iter, 1), np.float64)
    it = _load().or_hits(n2, _p(rp), _p(col), _p(val), tol, max_iter, _p(x), _p(res))
    if it < 0:
        raise ValueError("HITS: a half of the iterate sums to zero")
    return x, int(it), res[:it]


def rwr(csr, seeds, c=0.85, tol=0.0, max_iter=30):
    """RWR (Eq. 9) for every seed -> (R n x k, iterations, residuals it x k)."""
    n, _, rp, col, val = _csr(csr)
    seeds = np.ascontiguousarray(seeds, np.int32)
    k = len(seeds)
    R = np.empty((n, k), np.float64)
    res = np.zeros((max(max_iter, 1), k), np.float64)
    it = _load().or_rwr(n, _p(rp), _p(col), _p(val), _p(seeds), k, c, tol, max_iter, _p(R), _p(res))
    return R, int(it), res[:it]
