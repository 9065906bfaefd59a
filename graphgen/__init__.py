"""Seeded synthetic graphs and the matrices PageRank, HITS and RWR run on.

Input preparation shared by the oracle side and the GPU side.  Nothing here
computes any part of the SpMV method; see graphgen.c for the generators'
definitions.  All arrays are numpy (host) arrays:

    csr = (n_rows, n_cols, row_ptr int64[n_rows+1], col int32[nnz], val float32[nnz])
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, dbl, u64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        vp = ctypes.c_void_p
        lib.gg_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, vp, vp, vp]
        lib.gg_chung_lu.argtypes = [i32, i64, dbl, dbl, u64, vp, vp, vp]
        lib.gg_pagerank_csr.argtypes = [i64, i64, vp, vp, vp, vp, vp]
        lib.gg_hits_csr.argtypes = [i64, i64, vp, vp, vp, vp, vp]
        lib.gg_rwr_csr.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
        lib.gg_uniform_f32.argtypes = [i64, u64, vp]
        lib.gg_uniform_int.argtypes = [i64, u64, i64, vp]
        lib.gg_random_permutation.argtypes = [i64, u64, vp]
        for f in ("gg_rmat", "gg_chung_lu", "gg_pagerank_csr", "gg_hits_csr", "gg_rwr_csr"):
            getattr(lib, f).restype = ctypes.c_int
        lib.gg_uniform_f32.restype = None
        lib.gg_uniform_int.restype = None
        lib.gg_random_permutation.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """Directed simple graph on n nodes; edges sorted by (src, dst)."""
    n: int
    src: np.ndarray  # int32
    dst: np.ndarray  # int32

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def from_edges(n: int, src, dst) -> Graph:
    """Deduplicate and sort an explicit edge list (small graphs in tests)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    key = np.unique(src * n + dst)
    return Graph(n, (key // n).astype(np.int32), (key % n).astype(np.int32))


def rmat(scale: int, edge_factor: int = 16, a=0.57, b=0.19, c=0.19, seed: int = 0) -> Graph:
    """R-MAT graph, 2**scale nodes, edge_factor * 2**scale draws, duplicates removed."""
    lib = _load()
    m = int(edge_factor) << int(scale)
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    cnt = np.zeros(1, np.int64)
    rc = lib.gg_rmat(scale, m, a, b, c, seed, _p(src), _p(dst), _p(cnt))
    if rc != 0:
        raise RuntimeError("gg_rmat failed: %d" % rc)
    k = int(cnt[0])
    return Graph(1 << scale, src[:k].copy(), dst[:k].copy())


def chung_lu(log2n: int, n_edges: int, gamma: float = 2.1, cap: float = float(1 << 20),
             seed: int = 0) -> Graph:
    """Chung-Lu power-law graph with exactly n_edges distinct edges, ids permuted."""
    lib = _load()
    src = np.empty(n_edges, np.int32)
    dst = np.empty(n_edges, np.int32)
    cnt = np.zeros(1, np.int64)
    rc = lib.gg_chung_lu(log2n, n_edges, gamma, cap, seed, _p(src), _p(dst), _p(cnt))
    if rc != 0:
        raise RuntimeError("gg_chung_lu failed: %d" % rc)
    k = int(cnt[0])
    if k != n_edges:
        src, dst = src[:k].copy(), dst[:k].copy()
    return Graph(1 << log2n, src, dst)


def pagerank_matrix(g: Graph):
    """CSR of M = W^T: M[v][u] = fl32(1/outdeg(u)) for every edge u -> v."""
    lib = _load()
    rp = np.empty(g.n + 1, np.int64)
    col = np.empty(g.m, np.int32)
    val = np.empty(g.m, np.float32)
    rc = lib.gg_pagerank_csr(g.n, g.m, _p(g.src), _p(g.dst), _p(rp), _p(col), _p(val))
    if rc != 0:
        raise RuntimeError("gg_pagerank_csr failed: %d" % rc)
    return (g.n, g.n, rp, col, val)


def hits_matrix(g: Graph):
    """CSR of the 2n x 2n block matrix [[0, A^T], [A, 0]] with unit values."""
    lib = _load()
    rp = np.empty(2 * g.n + 1, np.int64)
    col = np.empty(2 * g.m, np.int32)
    val = np.empty(2 * g.m, np.float32)
    rc = lib.gg_hits_csr(g.n, g.m, _p(g.src), _p(g.dst), _p(rp), _p(col), _p(val))
    if rc != 0:
        raise RuntimeError("gg_hits_csr failed: %d" % rc)
    return (2 * g.n, 2 * g.n, rp, col, val)


def rwr_matrix(g: Graph):
    """CSR of the column-normalised adjacency of the symmetrised graph."""
    lib = _load()
    rp = np.empty(g.n + 1, np.int64)
    col = np.empty(2 * g.m, np.int32)
    val = np.empty(2 * g.m, np.float32)
    cnt = np.zeros(1, np.int64)
    rc = lib.gg_rwr_csr(g.n, g.m, _p(g.src), _p(g.dst), _p(rp), _p(col), _p(val), _p(cnt))
    if rc != 0:
        raise RuntimeError("gg_rwr_csr failed: %d" % rc)
    k = int(cnt[0])
    return (g.n, g.n, rp, col[:k].copy(), val[:k].copy())


def uniform_f32(n: int, seed: int) -> np.ndarray:
    """n floats uniform in [0,1), each a multiple of 2**-24."""
    out = np.empty(n, np.float32)
    _load().gg_uniform_f32(n, seed, _p(out))
    return out


def normal_f32(n: int, seed: int) -> np.ndarray:
    """n standard normal floats (Box-Muller on two uniform streams, FP64, then
    rounded to FP32); the edge features of the differentiable RWR."""
    u1 = uniform_f32(n, seed).astype(np.float64)
    u2 = uniform_f32(n, seed ^ 0x5DEECE66D).astype(np.float64)
    u1 = 1.0 - u1  # (0, 1]
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.float32)


def uniform_int(n: int, bound: int, seed: int) -> np.ndarray:
    out = np.empty(n, np.int64)
    _load().gg_uniform_int(n, seed, bound, _p(out))
    return out


def random_permutation(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, np.int32)
    _load().gg_random_permutation(n, seed, _p(out))
    return out


def rwr_seeds(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct seed nodes drawn uniformly from nodes with outdeg > 0."""
    outdeg = np.bincount(g.src, minlength=g.n)
    cand = np.nonzero(outdeg > 0)[0]
    perm = random_permutation(len(cand), seed)
    return cand[perm[:k]].astype(np.int32)


def random_csr(n_rows: int, n_cols: int, density: float, seed: int, values: str = "uniform",
               power: float | None = None):
    """Small random CSR matrix for tests (numpy Generator; not a graph model).

    values: "uniform" (U[0,1) floats), "dyadic" (from {+-1, +-1/2, +-1/4}) or "ones".
    power: if given, column j is drawn with weight (j+1)^-power (skewed columns).
    """
    rng = np.random.default_rng(seed)
    nnz_target = max(1, int(round(n_rows * n_cols * density)))
    if power is None:
        rows = rng.integers(0, n_rows, nnz_target)
        cols = rng.integers(0, n_cols, nnz_target)
    else:
        w = (np.arange(n_cols) + 1.0) ** (-power)
        w /= w.sum()
        cols = rng.choice(n_cols, nnz_target, p=w)
        wr = (np.arange(n_rows) + 1.0) ** (-power)
        wr /= wr.sum()
        rows = rng.permutation(n_rows)[rng.choice(n_rows, nnz_target, p=wr)]
        cols = rng.permutation(n_cols)[cols]
    key = np.unique(rows.astype(np.int64) * n_cols + cols)
    r = (key // n_cols).astype(np.int64)
    c = (key % n_cols).astype(np.int32)
    nnz = len(key)
    if values == "uniform":
        v = rng.random(nnz, dtype=np.float32)
    elif values == "dyadic":
        v = rng.choice(np.array([1, -1, 0.5, -0.5, 0.25, -0.25], np.float32), nnz)
    elif values == "ones":
        v = np.ones(nnz, np.float32)
    else:
        raise ValueError(values)
    rp = np.zeros(n_rows + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp)
    return (n_rows, n_cols, rp, c, v.astype(np.float32))
