"""Pins of the oracle's SpMV / SpMM against dense brute force, exact dyadic
arithmetic and invariants that the product y = A x must satisfy."""
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle


def dense(csr):
    n_rows, n_cols, rp, col, val = csr
    A = np.zeros((n_rows, n_cols))
    for i in range(n_rows):
        for k in range(rp[i], rp[i + 1]):
            A[i, col[k]] += float(val[k])
    return A


@pytest.mark.parametrize("shape,density,seed", [((1, 1), 1.0, 0), ((37, 53), 0.2, 1),
                                                 ((200, 120), 0.05, 2), ((256, 256), 0.1, 3)])
def test_spmv_matches_dense_bruteforce(shape, density, seed):
    csr = gg.random_csr(shape[0], shape[1], density, seed)
    x = gg.uniform_f32(shape[1], seed)
    y = oracle.spmv(csr, x)
    ref = dense(csr) @ x.astype(np.float64)
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-15)


def test_spmv_dyadic_is_exact():
    csr = gg.random_csr(60, 40, 0.3, 11, values="dyadic")
    n_rows, n_cols, rp, col, val = csr
    x = (np.arange(n_cols) % 7 - 3).astype(np.float32)
    y = oracle.spmv(csr, x)
    for i in range(n_rows):
        exact = sum((Fraction(float(val[k])) * Fraction(float(x[col[k]])) for k in range(rp[i], rp[i + 1])),
                    Fraction(0))
        assert Fraction(y[i]) == exact


def test_spmv_column_sum_identity_and_linearity():
    csr = gg.random_csr(300, 200, 0.03, 5, power=1.2)
    n_rows, n_cols, rp, col, val = csr
    x1 = gg.uniform_f32(n_cols, 1)
    x2 = gg.uniform_f32(n_cols, 2)
    colsum = np.bincount(col, weights=val.astype(np.float64), minlength=n_cols)
    y1 = oracle.spmv(csr, x1)
    assert abs(y1.sum() - colsum @ x1.astype(np.float64)) < 1e-10
    y12 = oracle.spmv(csr, (x1.astype(np.float64) + 3 * x2.astype(np.float64)))
    assert np.allclose(y12, y1 + 3 * oracle.spmv(csr, x2), rtol=1e-13, atol=1e-13)


def test_spmv_permutation_equivariance():
    csr = gg.random_csr(80, 80, 0.08, 9)
    n, _, rp, col, val = csr
    x = gg.uniform_f32(n, 3)
    P = gg.random_permutation(n, 17).astype(np.int64)  # new id of old i is P[i]
    inv = np.empty(n, np.int64)
    inv[P] = np.arange(n)
    # B = P A P^T : row P[i] of B is row i of A with columns relabelled
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = np.lexsort((P[col], P[rows]))
    r2, c2, v2 = P[rows][key], P[col][key], val[key]
    rp2 = np.concatenate([[0], np.cumsum(np.bincount(r2, minlength=n))])
    yB = oracle.spmv((n, n, rp2, c2.astype(np.int32), v2), x[inv])
    yA = oracle.spmv(csr, x)
    assert np.allclose(yB, yA[inv], rtol=1e-14, atol=0)


def test_column_stochastic_preserves_sum():
    g = gg.rmat(9, 8, seed=2)
    M = gg.pagerank_matrix(g)
    # remove dangling columns from x so the pin is exact up to FP32 values
    outdeg = np.bincount(g.src, minlength=g.n)
    x = gg.uniform_f32(g.n, 8) * (outdeg > 0)
    y = oracle.spmv(M, x)
    assert abs(y.sum() - x.astype(np.float64).sum()) <= 1e-6 * x.sum()


def test_absmv_and_rows():
    csr = gg.random_csr(50, 40, 0.2, 4, values="dyadic")
    x = (gg.uniform_f32(40, 1) - 0.5).astype(np.float32)
    A = dense(csr)
    assert np.allclose(oracle.absmv(csr, x), np.abs(A) @ np.abs(x.astype(np.float64)), rtol=1e-14)
    rows = np.array([0, 7, 49, 7])
    y, a = oracle.spmv_rows(csr, x, rows)
    assert np.allclose(y, (A @ x.astype(np.float64))[rows], rtol=1e-14, atol=1e-15)
    assert np.allclose(a, (np.abs(A) @ np.abs(x.astype(np.float64)))[rows], rtol=1e-14)


def test_spmm_matches_dense():
    csr = gg.random_csr(70, 90, 0.1, 6)
    X = np.stack([gg.uniform_f32(90, s) for s in range(5)], axis=1)
    Y = oracle.spmm(csr, X)
    assert np.allclose(Y, dense(csr) @ X.astype(np.float64), rtol=1e-13, atol=1e-15)


def test_empty_rows_and_columns():
    rp = np.array([0, 0, 2, 2, 3], np.int64)
    col = np.array([1, 3, 1], np.int32)
    val = np.array([2.0, -1.0, 0.5], np.float32)
    x = np.array([5, 1, 7, 3], np.float32)
    y = oracle.spmv((4, 4, rp, col, val), x)
    assert list(y) == [0.0, -1.0, 0.0, 0.5]
