"""Parity at the benchmark's full sizes, in the configuration bench.py times
(default build options): the 2^23-node / 2^27-edge Chung-Lu PageRank matrix,
the R-MAT 20 PageRank and HITS matrices and the symmetrised R-MAT 20 graph.
Every SpMV row is checked against the oracle, every format array bit for bit
against the reference builder, and PageRank, HITS, batched RWR and the
differentiable RWR's gradient against the full FP64 oracle."""
import os
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import ref_format as rf
from oracle.autotune import PerfTable

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # these tests need a GPU
    pytest.skip("no GPU", allow_module_level=True)

from paper_1103_2405_amd import DeviceCsr, TiledMatrix  # noqa: E402

TOL = 1e-5
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1103_2405_amd", "data", "perf_table_gfx950.txt")
FMT_KEYS = ["cperm", "rowmap", "tile_col_begin", "tile_col_end", "tile_nnz", "tile_wl", "tile_split", "tile_row_off",
            "rows_sorted", "rows_len", "wl_tile", "wl_layout", "wl_w", "wl_w_pad", "wl_h_pad", "wl_row_begin",
            "wl_n_rows", "wl_chunk", "wl_n_chunks", "wl_data_off", "wl_rowid_off", "idx", "rowid"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reference_default_format(csr):
    """The reference builder with the library's default options."""
    return rf.build(csr, W=1 << 23, table=PerfTable.load(TABLE), split_len=-1)


def assert_format_bit_exact(tm, csr):
    say("reference build of", len(csr[3]), "entries")
    ref = reference_default_format(csr)
    g = tm.export_format()
    assert g["T"] == ref["T"] and g["n_tiles_total"] == ref["n_tiles_total"] and g["nnz_pad"] == ref["nnz_pad"]
    for k in FMT_KEYS:
        a, b = np.asarray(g[k]), np.asarray(ref[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), k
    assert np.array_equal(g["val"].view(np.uint32), ref["val"].view(np.uint32)), "val"


def assert_spmv_all_rows(tm, csr, x):
    y = tm.spmv(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    ref = oracle.spmv(csr, x)
    bound = TOL * oracle.absmv(csr, x)
    err = np.abs(y - ref)
    bad = np.flatnonzero(err > bound)
    assert bad.size == 0, (bad[:5], err[bad[:5]], bound[bad[:5]])
    return y


@pytest.fixture(scope="module")
def cl23():
    g = gg.chung_lu(23, 1 << 27, gamma=2.1, cap=float(1 << 20), seed=23)
    return gg.pagerank_matrix(g)


@pytest.fixture(scope="module")
def cl23_handle(cl23):
    tm = TiledMatrix(DeviceCsr(cl23))
    yield tm
    tm.close()


def test_full_size_spmv_all_rows(cl23, cl23_handle):
    n, _, rp, col, val = cl23
    x = gg.uniform_f32(n, 101)
    y = assert_spmv_all_rows(cl23_handle, cl23, x)
    # sum y = sum over non-empty columns of x (the matrix is column-stochastic)
    clen = np.bincount(col, minlength=n)
    want = float(np.sum(x[clen > 0].astype(np.float64)))
    assert abs(float(y.sum()) - want) <= 1e-6 * want


def test_full_size_format_bit_exact(cl23, cl23_handle):
    assert_format_bit_exact(cl23_handle, cl23)


def test_full_size_pagerank_100_iterations(cl23, cl23_handle):
    p, it, _ = cl23_handle.pagerank(0.85, 0.0, 100)
    ref, _, _ = oracle.pagerank(cl23, 0.85, 0.0, 100)
    p = p.cpu().numpy().astype(np.float64)
    assert it == 100
    assert np.abs(p - ref).sum() <= 1e-6
    assert abs(p.sum() - 1.0) <= 1e-5


@pytest.fixture(scope="module")
def cl23_panels(cl23):
    # the configuration bench.py times: automatic row panels
    tm = TiledMatrix(DeviceCsr(cl23), panels=-1)
    yield tm
    tm.close()


def test_full_size_panels_spmv_all_rows_and_tile_order(cl23, cl23_panels):
    inf = cl23_panels.info()
    say("panels", inf["n_panels"], "column tiles", inf["n_col_tiles"], "rows", inf["panel_rows"],
        "tile width", inf["tile_width"])
    assert inf["n_panels"] > 1 and inf["n_col_tiles"] > 1
    # column tiles chosen from the device: a power of two of columns whose x
    # fills at most half an XCD's L2 (MI355X: 4 MB, so 2^19)
    W = inf["tile_width"]
    assert W >= 1 << 16 and W & (W - 1) == 0 and 8 * W <= 64 << 20
    n = cl23[0]
    x = gg.uniform_f32(n, 101)
    assert_spmv_all_rows(cl23_panels, cl23, x)
    # the one-launch panel pass gives the bits of the tile-by-tile launches
    xt = torch.from_numpy(x).cuda()
    ya, yb = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    cl23_panels.spmv_internal(xt, ya)
    cl23_panels.spmv_tiles(xt, yb)
    assert torch.equal(ya.view(torch.int32), yb.view(torch.int32))


def test_full_size_panels_pagerank_100_iterations(cl23, cl23_panels):
    # 99 iterations with the update fused into the panel pass, the last one separate
    p, it, _ = cl23_panels.pagerank(0.85, 0.0, 100)
    ref, _, _ = oracle.pagerank(cl23, 0.85, 0.0, 100)
    p = p.cpu().numpy().astype(np.float64)
    assert it == 100
    assert np.abs(p - ref).sum() <= 1e-6
    assert abs(p.sum() - 1.0) <= 1e-5


def test_rmat20_panels_format_bit_exact(rmat20):
    # automatic row panels on R-MAT 20: every array against the reference
    # builder given the parameters the handle reports
    csr = gg.pagerank_matrix(rmat20)
    with TiledMatrix(DeviceCsr(csr), panels=-1) as tm:
        inf = tm.info()
        f = tm.export_format()
        T = inf["n_dense_tiles"]
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        P = min(n_cu, -(-csr[0] // 2048))
        say("rmat20 panels", inf["n_panels"], "col tiles", inf["n_col_tiles"], "reference build ...")
        ref = rf.build(csr, W=inf["tile_width"], bounds=[int(v) for v in f["tile_col_end"][:T]],
                       wl=[512] * inf["n_tiles"], split_len=1024, panels=P, panel_rows=inf["panel_rows"],
                       panel_waves=inf["panel_waves"])
        assert f["n_tiles_total"] == ref["n_tiles_total"] and f["nnz_pad"] == ref["nnz_pad"]
        for k in FMT_KEYS + ["panel_begin"]:
            a, b = np.asarray(f[k]), np.asarray(ref[k])
            assert a.shape == b.shape and np.array_equal(a.astype(np.int64), b.astype(np.int64)), k
        assert np.array_equal(f["val"].view(np.uint32), ref["val"].view(np.uint32))
        assert_spmv_all_rows(tm, csr, gg.uniform_f32(rmat20.n, 7))


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


@pytest.fixture(scope="module")
def rmat20():
    return gg.rmat(20, 16, seed=20)


def test_rmat20_pagerank_matrix_spmv_format_and_50_iterations(rmat20):
    csr = gg.pagerank_matrix(rmat20)
    with TiledMatrix(DeviceCsr(csr)) as tm:
        assert_spmv_all_rows(tm, csr, gg.uniform_f32(rmat20.n, 101))
        assert_format_bit_exact(tm, csr)
        p, it, res = tm.pagerank(0.85, 0.0, 50)
        pref, _, rref = oracle.pagerank(csr, 0.85, 0.0, 50)
        d = np.abs(p.cpu().numpy().astype(np.float64) - pref).sum()
        say("rmat20 pagerank L1 diff", d)
        assert it == 50 and d <= 1e-6
        assert abs(res - rref[-1]) <= 1e-6


def test_rmat20_hits(rmat20):
    csr = gg.hits_matrix(rmat20)
    n = rmat20.n
    with TiledMatrix(DeviceCsr(csr)) as tm:
        a, h, it, _ = tm.hits(0.0, 30)
        x, _, _ = oracle.hits(csr, 0.0, 30)
        d = np.abs(a.cpu().numpy() - x[:n]).sum() + np.abs(h.cpu().numpy() - x[n:]).sum()
        say("rmat20 hits L1 diff", d)
        assert it == 30 and d <= 1e-6


def test_rmat20_rwr_gradient_matches_fp64_reference():
    # the benchmark's differentiable RWR at full size: symmetrised R-MAT 20,
    # 4 features per entry, 30 iterations, checkpoints every 6, 16 targets
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_oracle_rwr_grad import problem
    from oracle import rwr_grad as rg
    from paper_1103_2405_amd.rwr_grad import EdgeWeightedRWR
    n, rp, col, feats, theta, s, targets = problem(20, 16, 20)
    say("rmat20 gradient problem: n", n, "nnz", len(col))
    model = EdgeWeightedRWR((n, n, rp, col), feats, s, 0.85, 30, every=6)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    loss = -torch.log(model.scores(th)[torch.as_tensor(targets).cuda()].double()).sum()
    loss.backward()
    model.close()
    ref_loss, ref_grad, _ = rg.loss_and_grad(n, rp, col, feats, theta, s, targets, 0.85, 30)
    say("loss", loss.item(), ref_loss, "grad", th.grad.numpy(), ref_grad)
    assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss)
    assert np.linalg.norm(th.grad.numpy() - ref_grad) <= 1e-4 * np.linalg.norm(ref_grad)
