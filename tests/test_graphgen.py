"""Seeded input generators: determinism and the structure of the matrices."""
import numpy as np

import graphgen as gg


def test_rmat_deterministic_and_simple():
    g1 = gg.rmat(10, 8, seed=3)
    g2 = gg.rmat(10, 8, seed=3)
    g3 = gg.rmat(10, 8, seed=4)
    assert np.array_equal(g1.src, g2.src) and np.array_equal(g1.dst, g2.dst)
    assert not (len(g1.src) == len(g3.src) and np.array_equal(g1.src, g3.src))
    key = g1.src.astype(np.int64) * g1.n + g1.dst
    assert np.all(np.diff(key) > 0)  # sorted by (src, dst), no duplicates
    assert 0 < g1.m <= 8 * 1024
    assert g1.src.min() >= 0 and g1.dst.max() < g1.n


def test_rmat_skew():
    g = gg.rmat(12, 16, seed=12)
    outdeg = np.bincount(g.src, minlength=g.n)
    assert outdeg.max() > 20 * outdeg.mean()


def test_chung_lu_exact_count_and_skew():
    g = gg.chung_lu(12, 40000, gamma=2.1, cap=2000.0, seed=7)
    assert g.m == 40000
    key = g.src.astype(np.int64) * g.n + g.dst
    assert np.all(np.diff(key) > 0)
    outdeg = np.bincount(g.src, minlength=g.n)
    indeg = np.bincount(g.dst, minlength=g.n)
    assert outdeg.max() > 20 * outdeg.mean() and indeg.max() > 20 * indeg.mean()
    g2 = gg.chung_lu(12, 40000, gamma=2.1, cap=2000.0, seed=7)
    assert np.array_equal(g.src, g2.src) and np.array_equal(g.dst, g2.dst)


def test_pagerank_matrix_is_column_stochastic():
    g = gg.rmat(10, 8, seed=1)
    n, _, rp, col, val = gg.pagerank_matrix(g)
    outdeg = np.bincount(g.src, minlength=n)
    colsum = np.bincount(col, weights=val.astype(np.float64), minlength=n)
    nz = outdeg > 0
    assert np.all(np.abs(colsum[nz] - 1.0) <= outdeg[nz] * 2.0 ** -24)
    assert np.all(colsum[~nz] == 0)
    # entry M[v][u] exists iff edge u -> v
    rows = np.repeat(np.arange(n), np.diff(rp))
    k1 = np.sort(col.astype(np.int64) * n + rows)
    k2 = g.src.astype(np.int64) * n + g.dst
    assert np.array_equal(k1, k2)
    for i in range(n):
        assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)


def test_hits_matrix_blocks():
    g = gg.from_edges(4, [0, 0, 1, 3], [1, 2, 2, 0])
    N, _, rp, col, val = gg.hits_matrix(g)
    B = np.zeros((N, N))
    for i in range(N):
        B[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    A = np.zeros((4, 4))
    A[g.src, g.dst] = 1
    assert np.array_equal(B[:4, 4:], A.T) and np.array_equal(B[4:, :4], A)
    assert not B[:4, :4].any() and not B[4:, 4:].any()


def test_rwr_matrix_symmetrised_column_normalised():
    g = gg.from_edges(5, [0, 1, 1, 2, 3, 3], [1, 0, 2, 2, 4, 1])
    n, _, rp, col, val = gg.rwr_matrix(g)
    S = np.zeros((n, n))
    for i in range(n):
        S[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    P = (S != 0)
    assert np.array_equal(P, P.T)
    deg = P.sum(axis=0)
    for j in range(n):
        if deg[j]:
            assert np.allclose(S[P[:, j], j], np.float32(1) / np.float32(deg[j]))
    assert P[2, 2]  # self-loop kept once


def test_uniform_f32_is_24bit():
    x = gg.uniform_f32(1000, 5)
    assert x.dtype == np.float32 and x.min() >= 0 and x.max() < 1
    assert np.all((x * 2.0 ** 24) == np.floor(x * 2.0 ** 24))
    assert np.array_equal(x, gg.uniform_f32(1000, 5))
