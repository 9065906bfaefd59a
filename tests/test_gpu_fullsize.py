"""Parity at the benchmark's full sizes, in the configuration bench.py times
(default build options): the 2^23-node / 2^27-edge Chung-Lu PageRank matrix
and the symmetrised R-MAT 20 graph.  SpMV is checked on sampled rows the
oracle computes one by one (plus the longest and the empty rows) and by an
identity over all rows; PageRank and batched RWR against the full oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # these tests need a GPU
    pytest.skip("no GPU", allow_module_level=True)

from paper_1103_2405_amd import DeviceCsr, TiledMatrix  # noqa: E402

TOL = 1e-5


@pytest.fixture(scope="module")
def cl23():
    g = gg.chung_lu(23, 1 << 27, gamma=2.1, cap=float(1 << 20), seed=23)
    return gg.pagerank_matrix(g)


@pytest.fixture(scope="module")
def cl23_handle(cl23):
    tm = TiledMatrix(DeviceCsr(cl23))
    yield tm
    tm.close()


def test_full_size_spmv_sampled_rows(cl23, cl23_handle):
    n, _, rp, col, val = cl23
    x = gg.uniform_f32(n, 101)
    y = cl23_handle.spmv(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    lens = np.diff(rp)
    rows = np.unique(np.concatenate([
        gg.uniform_int(200000, n, 7),                 # uniform sample
        np.argsort(-lens, kind="stable")[:2000],      # the heaviest rows (split across wavefronts)
        np.flatnonzero(lens == 0)[:2000],             # empty rows
        [0, n - 1]]))
    ref, absref = oracle.spmv_rows(cl23, x, rows)
    err = np.abs(y[rows] - ref)
    bad = np.flatnonzero(err > TOL * absref)
    assert bad.size == 0, (rows[bad[:5]], err[bad[:5]], absref[bad[:5]])
    # all rows: sum y = sum over non-empty columns of x (the matrix is column-stochastic)
    clen = np.bincount(col, minlength=n)
    want = float(np.sum(x[clen > 0].astype(np.float64)))
    assert abs(float(y.sum()) - want) <= 1e-6 * want


def test_full_size_pagerank_100_iterations(cl23, cl23_handle):
    p, it, _ = cl23_handle.pagerank(0.85, 0.0, 100)
    ref, _, _ = oracle.pagerank(cl23, 0.85, 0.0, 100)
    p = p.cpu().numpy().astype(np.float64)
    assert it == 100
    assert np.abs(p - ref).sum() <= 1e-6
    assert abs(p.sum() - 1.0) <= 1e-5


@pytest.fixture(scope="module")
def rmat20_rwr():
    g = gg.rmat(20, 16, seed=20)
    W = gg.rwr_matrix(g)
    tm = TiledMatrix(DeviceCsr(W))
    yield g, W, tm
    tm.close()


def test_full_size_batched_rwr_k32(rmat20_rwr):
    g, W, tm = rmat20_rwr
    seeds = gg.rwr_seeds(g, 32, 40)
    R, it, _ = tm.rwr(seeds, 0.85, 0.0, 20)
    ref, _, _ = oracle.rwr(W, seeds, 0.85, 0.0, 20)
    d = np.abs(R.cpu().numpy().astype(np.float64) - ref).sum(axis=0)
    assert np.all(d <= 1e-6), d.max()


def test_full_size_single_query_rwr_fused_equals_separate(rmat20_rwr):
    # the single-vector tile kernel with the restart fused in (row slices at
    # this size) against iterations that all read the change (no fused step)
    g, W, tm = rmat20_rwr
    seeds = gg.rwr_seeds(g, 1, 40)
    a, it, ra = tm.rwr(seeds, 0.85, 1e-7, 500, 1)
    b, it2, rb = tm.rwr(seeds, 0.85, 0.0, it)
    assert it2 == it and ra == rb
    assert torch.equal(a, b)
    ref, _, _ = oracle.rwr(W, seeds, 0.85, 0.0, it)
    assert np.abs(b.cpu().numpy().astype(np.float64) - ref).sum() <= 1e-6
