"""GPU parity: the HIP library against the oracle, through the C ABI.

  format   every metadata array, every packed index and every packed value
           bit-exact against the reference builder
  SpMV     |y - y_ref|_i <= 1e-5 (|A| |x|)_i per entry (FP64 oracle), and
           bit-exact on dyadic inputs (every order of summation is exact)
  drivers  L1 distance of iterates at equal iteration counts <= 1e-6
"""
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

from paper_1103_2405_amd import TcError, TiledMatrix, DeviceCsr, csr_spmv  # noqa: E402
from paper_1103_2405_amd import tc as tcmod  # noqa: E402

TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


FMT_KEYS = ["cperm", "rowmap", "tile_col_begin", "tile_col_end", "tile_nnz", "tile_wl", "tile_split", "tile_row_off",
            "rows_sorted", "rows_len", "wl_tile", "wl_layout", "wl_w", "wl_w_pad", "wl_h_pad", "wl_row_begin",
            "wl_n_rows", "wl_chunk", "wl_n_chunks", "wl_data_off", "wl_rowid_off", "idx", "rowid"]


def assert_same_format(g, r):
    assert g["T"] == r["T"] and g["n_tiles_total"] == r["n_tiles_total"] and g["nnz_pad"] == r["nnz_pad"]
    for k in FMT_KEYS:
        a, b = np.asarray(g[k]), np.asarray(r[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), k
    assert np.array_equal(g["val"].view(np.uint32), r["val"].view(np.uint32)), "val"


def build_both(csr, W, wl=None, S=64, split_len=-1, n_tiles=-1, camping_pad=False, table_path=None,
               max_act_warp=8192, xcd_groups=0, kernel="composite", bounds=None):
    say("build", csr[0], csr[1], len(csr[3]), "W", W, "wl", wl if not isinstance(wl, list) else wl[:3], "S", S,
        "split", split_len)
    wl_list = wl if wl is None or isinstance(wl, list) else [wl] * 4096
    ref = rf.build(csr, W=W, n_tiles=n_tiles, wl=wl_list, S=S, split_len=split_len, camping_pad=camping_pad,
                   table=PerfTable.load(table_path) if table_path else None, max_act_warp=max_act_warp,
                   xcd_groups=xcd_groups, coo=kernel == "coo", bounds=bounds)
    gm = TiledMatrix(csr, tile_width=W, n_tiles=n_tiles, wl=wl, wave=S, split_len=split_len,
                     camping_pad=camping_pad, perf_table=table_path, max_act_warp=max_act_warp,
                     xcd_groups=xcd_groups, kernel=kernel, tile_bounds=bounds)
    return gm, ref


def check_spmv(gm, csr, x, exact=False):
    xt = torch.from_numpy(x).cuda()
    y = gm.spmv(xt).cpu().numpy().astype(np.float64)
    ref = oracle.spmv(csr, x)
    if exact:
        assert np.array_equal(y, ref)
        return
    bound = TOL * oracle.absmv(csr, x)
    err = np.abs(y - ref)
    bad = np.flatnonzero(err > bound)
    assert bad.size == 0, (bad[:10], err[bad[:10]], bound[bad[:10]])


# ------------------------------------------------------------------ format
def test_format_figure1_example():
    from test_ref_format import load_fig1
    csr, p, expect = load_fig1()
    gm, ref = build_both(csr, W=p["W"], wl=[p["WL"]] * 3, S=p["S"], split_len=0)
    assert_same_format(gm.export_format(), ref)
    check_spmv(gm, csr, np.arange(1, 9, dtype=np.float32), exact=True)


@pytest.mark.parametrize("seed,n,density,W,wl,S,split", [
    (0, 300, 0.03, 16, 64, 64, 0),
    (1, 300, 0.03, 7, 12, 4, 0),
    (2, 500, 0.02, 32, 200, 64, 40),
    (3, 200, 0.05, 5, 3, 2, 6),
    (4, 1000, 0.01, 100, 500, 64, 100),
    (5, 2000, 0.005, 256, 1000, 64, 64),
])
def test_format_bit_exact_small(seed, n, density, W, wl, S, split):
    csr = gg.random_csr(n, n, density, seed, power=1.1)
    gm, ref = build_both(csr, W=W, wl=wl, S=S, split_len=split)
    assert_same_format(gm.export_format(), ref)


def test_format_rectangular_and_camping_pad():
    csr = gg.random_csr(300, 900, 0.01, 7, power=1.0)
    gm, ref = build_both(csr, W=64, wl=256, S=64, split_len=32, camping_pad=True)
    g = gm.export_format()
    assert not g["relabel"]
    assert_same_format(g, ref)
    check_spmv(gm, csr, gg.uniform_f32(900, 1))


def test_format_square_without_relabel_several_tiles():
    # rows keep their ids: the entries stay in CSR order through the tile
    # passes and the segment sort skips the row bits, as with relabelled rows
    csr = gg.random_csr(1500, 1500, 0.01, 21, power=1.1)
    ref = rf.build(csr, W=128, wl=[300] * 4096, S=64, split_len=64, relabel=False)
    gm = TiledMatrix(csr, tile_width=128, wl=300, wave=64, split_len=64, relabel=0)
    g = gm.export_format()
    assert not g["relabel"] and ref["n_tiles_total"] > 1
    assert_same_format(g, ref)
    check_spmv(gm, csr, gg.uniform_f32(1500, 22))
    gm.close()


def test_format_rmat14_several_tiles():
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    for W, wl, split in [(1024, 2048, 512), (4096, 512, 8192), (1 << 14, 4096, 256), (2048, 300, -1)]:
        gm, ref = build_both(csr, W=W, wl=wl, split_len=split)
        assert_same_format(gm.export_format(), ref)
        check_spmv(gm, csr, gg.uniform_f32(g.n, 101))


def _write_table(path):
    # a synthetic table (not measured): favours wide rows and tall columns
    with open(path, "w") as f:
        for kind, scale in (("dense", 1.0), ("sparse", 0.8)):
            for lw in range(16):
                for lh in range(16):
                    w, h = 2 ** lw, 2 ** lh
                    v = int(1e6 * scale * (w * h) / (w * h + 512 + 40 * min(w, h)))
                    f.write("%s %d %d %d\n" % (kind, lw, lh, max(v, 1)))


def test_autotuned_workload_sizes_match_reference(tmp_path):
    path = str(tmp_path / "table.txt")
    _write_table(path)
    g = gg.rmat(13, 16, seed=3)
    csr = gg.pagerank_matrix(g)
    for split, mw in ((1024, 64), (-1, 128)):
        gm, ref = build_both(csr, W=1024, wl=None, split_len=split, table_path=path, max_act_warp=mw)
        fmt = gm.export_format()
        assert list(fmt["tile_wl"]) == list(ref["tile_wl"])
        assert len(set(ref["tile_wl"])) > 1
        assert_same_format(fmt, ref)
        check_spmv(gm, csr, gg.uniform_f32(g.n, 5))


@pytest.mark.parametrize("W,groups,split", [(1024, 8, -1), (256, 3, 64), (4096, 8, 0)])
def test_xcd_schedule_format_and_products(W, groups, split):
    """XCD schedule: head tile plus column ranges of equal entries, bit-exact
    format; products, SpMM and PageRank through the concurrent pinned pass."""
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    gm, ref = build_both(csr, W=W, wl=512, split_len=split, xcd_groups=groups)
    fmt = gm.export_format()
    assert fmt["xcd_groups"] == groups and fmt["n_tiles_total"] == groups + 1
    assert_same_format(fmt, ref)
    x = gg.uniform_f32(g.n, 7)
    check_spmv(gm, csr, x)
    X = np.stack([gg.uniform_f32(g.n, 20 + q) for q in range(4)], axis=1)
    Y = gm.spmm(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Y - oracle.spmm(csr, X)) <= TOL * oracle.spmm(
        (csr[0], csr[1], csr[2], csr[3], np.abs(csr[4])), np.abs(X)))
    p, it, res = gm.pagerank(0.85, 0.0, 30)
    pref, _, _ = oracle.pagerank(csr, 0.85, 0.0, 30)
    assert np.abs(p.cpu().numpy().astype(np.float64) - pref).sum() <= 1e-6


def test_xcd_schedule_dyadic_bit_exact():
    csr = gg.random_csr(3000, 3000, 0.004, 5, values="dyadic", power=1.2)
    x = ((np.arange(3000) * 5) % 7 - 3).astype(np.float32)
    check_spmv(TiledMatrix(csr, tile_width=64, wl=300, split_len=16, xcd_groups=8), csr, x, exact=True)


# ------------------------------------------------------------------- SpMV
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spmv_dyadic_bit_exact(seed):
    csr = gg.random_csr(3000, 3000, 0.004, seed, values="dyadic", power=1.2)
    x = ((np.arange(3000) * 7 + seed) % 7 - 3).astype(np.float32)
    gm = TiledMatrix(csr, tile_width=256, wl=300, split_len=16)
    check_spmv(gm, csr, x, exact=True)


def test_spmv_rmat14_default_options():
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    gm = TiledMatrix(csr)
    say(gm.info())
    check_spmv(gm, csr, gg.uniform_f32(g.n, 101))


def test_spmv_signed_values_and_ragged_tiles():
    csr = gg.random_csr(5000, 4000, 0.003, 9, power=1.3)
    n_rows, n_cols, rp, col, val = csr
    val = (val - 0.5).astype(np.float32)
    csr = (n_rows, n_cols, rp, col, val)
    x = (gg.uniform_f32(n_cols, 2) * 2 - 1).astype(np.float32)
    for W in (100, 999, 4000):
        check_spmv(TiledMatrix(csr, tile_width=W, wl=256, split_len=64), csr, x)


def test_spmm_matches_oracle():
    g = gg.rmat(12, 16, seed=4)
    csr = gg.rwr_matrix(g)
    gm = TiledMatrix(csr, tile_width=512, wl=1024, split_len=256)
    for k in (1, 3, 8, 13, 32, 64, 100):
        X = np.stack([gg.uniform_f32(g.n, 10 + q) for q in range(k)], axis=1)
        Y = gm.spmm(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
        ref = oracle.spmm(csr, X)
        bound = TOL * oracle.spmm((csr[0], csr[1], csr[2], csr[3], np.abs(csr[4])), np.abs(X))
        assert np.all(np.abs(Y - ref) <= bound), k


def _heavy_rows_csr(n, heavy, heavy_len, light_len, seed, dyadic):
    """n x n CSR whose first `heavy` rows hold heavy_len distinct columns and
    every other row light_len; dyadic values when asked."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        m = heavy_len if i < heavy else int(rng.integers(0, light_len + 1))
        rows.append(np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32))
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate(rows).astype(np.int32)
    if dyadic:
        val = rng.choice(np.array([1, -1, 0.5, -0.5, 0.25, -0.25], np.float32), size=col.size)
    else:
        val = rng.random(col.size, dtype=np.float32)
    return (n, n, rp, col, val.astype(np.float32))


@pytest.mark.parametrize("W,split", [(4096, 1280), (1024, 256), (4096, 0)])
def test_spmm_heavy_rows_in_pieces(W, split):
    # rows of 2500 entries: with split 1280 every chunk is summed in three
    # 512-entry pieces; with 0 the rows stay whole (row-major, all groups)
    csr = _heavy_rows_csr(3000, 5, 2500, 6, 17, dyadic=False)
    gm = TiledMatrix(csr, tile_width=W, split_len=split)
    for k in (1, 2, 7, 32, 64, 65, 130):
        X = np.stack([gg.uniform_f32(csr[1], 40 + q) for q in range(k)], axis=1)
        Y = gm.spmm(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
        ref = oracle.spmm(csr, X)
        bound = TOL * oracle.spmm((csr[0], csr[1], csr[2], csr[3], np.abs(csr[4])), np.abs(X))
        assert np.all(np.abs(Y - ref) <= bound), (W, split, k)


def test_spmm_dyadic_bit_exact():
    # dyadic values and small-integer X: every summation order is exact, so
    # each column of Y must equal the oracle bit for bit
    csr = _heavy_rows_csr(3000, 4, 2200, 9, 23, dyadic=True)
    gm = TiledMatrix(csr, tile_width=1024, split_len=1024)
    rng = np.random.default_rng(5)
    for k in (1, 9, 64, 70):
        X = rng.integers(-8, 9, size=(csr[1], k)).astype(np.float32)
        Y = gm.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
        assert np.array_equal(Y.astype(np.float64), oracle.spmm(csr, X)), k


def test_csr_baseline_matches_oracle():
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    x = gg.uniform_f32(g.n, 101)
    y = csr_spmv(DeviceCsr(csr), torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(y - oracle.spmv(csr, x)) <= TOL * oracle.absmv(csr, x))


# ------------------------------------------------------------ edge cases
def test_empty_and_tiny_matrices():
    # no entries at all
    csr = (5, 7, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    gm = TiledMatrix(csr, tile_width=4)
    y = gm.spmv(torch.ones(7, device="cuda"))
    assert torch.all(y == 0)
    # 1 x 1
    csr = (1, 1, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([2.5], np.float32))
    gm = TiledMatrix(csr, tile_width=1)
    assert gm.spmv(torch.full((1,), 2.0, device="cuda")).item() == 5.0
    # a single dense row (one heavy row split into many chunks)
    n = 20000
    csr = (3, n, np.array([0, 0, n, n], np.int64), np.arange(n, dtype=np.int32), gg.uniform_f32(n, 3))
    check_spmv(TiledMatrix(csr, tile_width=4096, split_len=1000), csr, gg.uniform_f32(n, 4))


def test_invalid_csr_rejected():
    bad_rp = (3, 3, np.array([0, 2, 1, 3], np.int64), np.array([0, 1, 2], np.int32), np.ones(3, np.float32))
    with pytest.raises(TcError) as e:
        TiledMatrix(bad_rp)
    assert e.value.status == tcmod.TC_EINVAL
    bad_col = (2, 2, np.array([0, 1, 2], np.int64), np.array([0, 2], np.int32), np.ones(2, np.float32))
    with pytest.raises(TcError) as e:
        TiledMatrix(bad_col)
    assert e.value.status == tcmod.TC_EINVAL
    bad_end = (2, 2, np.array([0, 1, 1], np.int64), np.array([0, 1], np.int32), np.ones(2, np.float32))
    with pytest.raises(TcError):
        TiledMatrix(bad_end)


def test_aliasing_rejected():
    csr = gg.random_csr(50, 50, 0.1, 1)
    gm = TiledMatrix(csr, tile_width=16)
    x = torch.ones(50, device="cuda")
    with pytest.raises(TcError):
        gm.spmv(x, x)


# ---------------------------------------------------------------- drivers
def test_pagerank_rmat14_50_iterations():
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    gm = TiledMatrix(csr)
    p, it, res = gm.pagerank(0.85, 0.0, 50)
    pref, _, rref = oracle.pagerank(csr, 0.85, 0.0, 50)
    assert it == 50
    d = np.abs(p.cpu().numpy().astype(np.float64) - pref).sum()
    say("pagerank L1 diff", d, "resid", res, rref[-1])
    assert d <= 1e-6
    assert abs(res - rref[-1]) <= 1e-6


@pytest.mark.parametrize("split", [-1, 64])
def test_pagerank_fused_update_equals_separate_update(split):
    # with the change read every iteration no step is fused; with a fixed
    # count every step but the last is: the iterates must agree bit for bit
    # (rows without entries, dangling columns and split rows included)
    g = gg.rmat(13, 8, seed=21)
    csr = gg.pagerank_matrix(g)
    assert np.any(np.diff(csr[2]) == 0) and np.any(np.bincount(csr[3], minlength=csr[1]) == 0)
    gm = TiledMatrix(csr, split_len=split)
    assert gm.info()["n_tiles"] == 1
    a, it, ra = gm.pagerank(0.85, 1e-7, 300, check_every=1)
    b, it2, rb = gm.pagerank(0.85, 0.0, it)
    assert it2 == it and ra == rb
    assert torch.equal(a, b)
    pref, _, _ = oracle.pagerank(csr, 0.85, 0.0, it)
    assert np.abs(b.cpu().numpy() - pref).sum() <= 1e-6


def test_pagerank_converges_to_tolerance():
    g = gg.rmat(12, 16, seed=1)
    csr = gg.pagerank_matrix(g)
    gm = TiledMatrix(csr, tile_width=256)
    p, it, res = gm.pagerank(0.85, 1e-6, 500, check_every=5)
    assert res <= 1e-6 and it % 5 == 0
    pref, itr, _ = oracle.pagerank(csr, 0.85, 0.0, it)
    assert np.abs(p.cpu().numpy() - pref).sum() <= 1e-6
    with pytest.raises(tcmod.NotConverged):
        gm.pagerank(0.85, 1e-12, 3)


def test_hits_matches_oracle():
    g = gg.rmat(12, 16, seed=7)
    csr = gg.hits_matrix(g)
    gm = TiledMatrix(csr, tile_width=1024)
    a, h, it, res = gm.hits(0.0, 30)
    x, _, rref = oracle.hits(csr, 0.0, 30)
    n = g.n
    d = np.abs(a.cpu().numpy() - x[:n]).sum() + np.abs(h.cpu().numpy() - x[n:]).sum()
    say("hits L1 diff", d)
    assert d <= 1e-6
    empty = gg.hits_matrix(gg.from_edges(4, [], []))
    with pytest.raises(TcError):
        TiledMatrix(empty).hits(0.0, 2)


@pytest.mark.parametrize("W", [1024, 0])  # several tiles; one tile (restart fused into the SpMM)
def test_rwr_matches_oracle(W):
    g = gg.rmat(12, 16, seed=8)
    csr = gg.rwr_matrix(g)
    gm = TiledMatrix(csr, tile_width=W)
    seeds = gg.rwr_seeds(g, 40, 40)
    for k in (1, 5, 32, 37, 40):  # 37, 40: right-hand sides in two passes
        R, it, res = gm.rwr(seeds[:k], 0.85, 0.0, 30)
        Rref, _, rr = oracle.rwr(csr, seeds[:k], 0.85, 0.0, 30)
        d = np.abs(R.cpu().numpy() - Rref).sum(axis=0)
        say("rwr L1 diff per column", d)
        assert np.all(d <= 1e-6)


@pytest.mark.parametrize("split", [-1, 64])
def test_rwr_fused_restart_equals_separate_update(split):
    # with the change read every iteration no step is fused; with a fixed
    # count every step but the last is: the iterates must agree bit for bit.
    # A seed on a node without edges exercises the rows no workload writes.
    g = gg.rmat(12, 8, seed=5)
    csr = gg.rwr_matrix(g)
    empty = np.flatnonzero(np.diff(csr[2]) == 0)
    assert empty.size > 0
    seeds = [int(v) for v in gg.rwr_seeds(g, 39, 3)] + [int(empty[0])]
    gm = TiledMatrix(csr, split_len=split)
    assert gm.info()["n_tiles"] == 1
    # 4-wide SpMM (40: two passes), 1-wide SpMM, the single-vector tile kernel
    for k in (40, 8, 3, 1):
        a, it, ra = gm.rwr(seeds[-k:], 0.85, 1e-7, 500, 1)
        b, it2, rb = gm.rwr(seeds[-k:], 0.85, 0.0, it)
        assert it2 == it and ra == rb
        assert torch.equal(a, b), k
        ref, _, _ = oracle.rwr(csr, seeds[-k:], 0.85, 0.0, it)
        assert np.all(np.abs(b.cpu().numpy() - ref).sum(axis=0) <= 1e-6)


# ------------------------------------------------------------ several graphs per launch
def _multi_set(one_tile=False):
    mats, csrs, seeds = [], [], []
    for gi in range(6):
        g = gg.rmat(8 + gi % 4, 4 + 3 * gi, seed=700 + gi)
        csr = gg.rwr_matrix(g)
        # mixed formats: several tiles, split rows, one tile (all one tile:
        # the restart is fused into the products)
        W = 128 if gi % 2 and not one_tile else 0
        split = 64 if gi % 3 == 0 else -1
        mats.append(TiledMatrix(csr, tile_width=W, split_len=split))
        csrs.append(csr)
        seeds.append(int(gg.rwr_seeds(g, 1, 50 + gi)[0]))
    return mats, csrs, seeds


@pytest.mark.parametrize("one_tile", [False, True])
def test_rwr_multi_matches_oracle_and_single_graph_driver(one_tile):
    from paper_1103_2405_amd import rwr_multi
    mats, csrs, seeds = _multi_set(one_tile)
    eager, it, res = rwr_multi(mats, seeds, 0.85, 0.0, 30, 1, graph=False)
    assert it == 30
    for m, csr, s, r in zip(mats, csrs, seeds, eager):
        ref, _, _ = oracle.rwr(csr, [s], 0.85, 0.0, 30)
        d = np.abs(r.cpu().numpy() - ref[:, 0]).sum()
        say("multi rwr L1 diff", d)
        assert d <= 1e-6
        # the same kernels as the single-graph driver: identical iterates
        one, _, _ = m.rwr([s], 0.85, 0.0, 30)
        assert torch.equal(one[:, 0], r)
    # the HIP graph replays give the eager result, call after call
    for rep in range(3):
        got, it2, _ = rwr_multi(mats, seeds, 0.85, 0.0, 30, 10, graph=True)
        assert it2 == 30
        for a, b in zip(got, eager):
            assert torch.equal(a, b), rep
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays


@pytest.mark.parametrize("one_tile,every", [(False, 5), (True, 5), (True, 4), (True, 1)])
def test_rwr_multi_tolerance_and_empty(one_tile, every):
    # with one tile per graph, a captured chunk of `every` iterations holds
    # every - 1 fused steps: an odd count flips the buffers, so replays
    # alternate between the two captured graphs
    from paper_1103_2405_amd import rwr_multi
    mats, csrs, seeds = _multi_set(one_tile)
    out, it, res = rwr_multi(mats, seeds, 0.85, 1e-6, 500, every, graph=True)
    assert it % every == 0 and res.max() <= 1e-6
    eager, it2, res2 = rwr_multi(mats, seeds, 0.85, 1e-6, 500, every, graph=False)
    assert it2 == it and np.array_equal(res, res2)
    for m, csr, s, r, e in zip(mats, csrs, seeds, out, eager):
        assert torch.equal(r, e)
        one, _, _ = m.rwr([s], 0.85, 0.0, it)
        assert torch.equal(one[:, 0], r)
        ref, _, _ = oracle.rwr(csr, [s], 0.85, 0.0, it)
        assert np.abs(r.cpu().numpy() - ref[:, 0]).sum() <= 1e-6
    out, it, res = rwr_multi([], [], 0.85, 0.0, 30, 1)
    assert out == [] and it == 0
    with pytest.raises(TcError):
        rwr_multi(mats[:2], [seeds[0], -1], 0.85, 0.0, 5, 1)


def test_rwr_multi_with_a_graph_larger_than_lds():
    # every graph one tile (the fused restart), one of them with more columns
    # than an LDS holds and one with split rows: the same bits as the
    # single-graph driver, within the FP32 bound of the oracle
    from paper_1103_2405_amd import rwr_multi
    mats, csrs, seeds = [], [], []
    for gi, (sc, ef) in enumerate([(16, 8), (9, 6), (12, 20), (10, 3)]):
        g = gg.rmat(sc, ef, seed=900 + gi)
        csr = gg.rwr_matrix(g)
        mats.append(TiledMatrix(csr, split_len=64 if gi == 2 else -1))
        csrs.append(csr)
        seeds.append(int(gg.rwr_seeds(g, 1, 950 + gi)[0]))
    assert mats[0].info()["n_tiles"] == 1 and csrs[0][1] > 40960
    for graph in (False, True):
        out, it, _ = rwr_multi(mats, seeds, 0.85, 0.0, 20, 5, graph=graph)
        assert it == 20
        for m, csr, s, r in zip(mats, csrs, seeds, out):
            one, _, _ = m.rwr([s], 0.85, 0.0, 20)
            assert torch.equal(one[:, 0], r)
            ref, _, _ = oracle.rwr(csr, [s], 0.85, 0.0, 20)
            d = np.abs(r.cpu().numpy() - ref[:, 0]).sum()
            say("lds multi rwr n", csr[0], "L1 diff", d)
            assert d <= 1e-5
    for m in mats:
        m.close()


@pytest.mark.parametrize("W,split,panels", [(0, -1, 0), (0, 64, 0), (1024, 64, 0), (1024, 64, -1)])
def test_refresh_values_equals_fresh_build(W, split, panels):
    # a handle built with the value map and then given new values holds
    # exactly what a build from the new values holds
    g = gg.rmat(12, 8, seed=31)
    n, _, rp, col, val = gg.pagerank_matrix(g)
    val2 = gg.uniform_f32(len(col), 32)
    kw = dict(tile_width=W, split_len=split, panels=panels)
    tm = TiledMatrix((n, n, rp, col, val), value_map=True, **kw)
    same = TiledMatrix((n, n, rp, col, val), **kw)
    fresh = TiledMatrix((n, n, rp, col, val2), **kw)
    a0, s0 = tm.export_format(), same.export_format()
    for key in ("idx", "val", "rowid"):
        assert np.array_equal(a0[key].view(np.uint32), s0[key].view(np.uint32)), key
    tm.refresh_values(torch.from_numpy(val2).cuda())
    a, b = tm.export_format(), fresh.export_format()
    for key in ("idx", "val", "rowid"):
        assert np.array_equal(a[key].view(np.uint32), b[key].view(np.uint32)), key
    x = torch.from_numpy(gg.uniform_f32(n, 33)).cuda()
    assert torch.equal(tm.spmv(x), fresh.spmv(x))
    with pytest.raises(TcError):
        fresh.refresh_values(torch.from_numpy(val2).cuda())
    for m in (tm, same, fresh):
        m.close()


# ------------------------------------------------------------ differentiable RWR
def test_csr_transpose_bit_exact():
    g = gg.rmat(11, 8, seed=12)
    n, _, rp, col, val = gg.pagerank_matrix(g)
    A = DeviceCsr((n, n, rp, col, val))
    rpT = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    colT = torch.empty(len(col), dtype=torch.int32, device="cuda")
    valT = torch.empty(len(col), dtype=torch.float32, device="cuda")
    permT = torch.empty(len(col), dtype=torch.int32, device="cuda")
    import ctypes
    lib = tcmod.load_library()
    c = A.c()
    assert lib.tc_csr_transpose(ctypes.byref(c), ctypes.c_void_p(rpT.data_ptr()), ctypes.c_void_p(colT.data_ptr()),
                                ctypes.c_void_p(valT.data_ptr()), ctypes.c_void_p(permT.data_ptr()), None) == 0
    rows = np.repeat(np.arange(n), np.diff(rp))
    order = np.lexsort((rows, col))  # by column, then row: a stable sort by column
    assert np.array_equal(permT.cpu().numpy(), order)
    assert np.array_equal(colT.cpu().numpy(), rows[order])
    assert np.array_equal(valT.cpu().numpy(), val[order])
    assert np.array_equal(rpT.cpu().numpy(), np.concatenate([[0], np.cumsum(np.bincount(col, minlength=n))]))


def test_gather_rows_bit_exact_and_index_check():
    import ctypes
    lib = tcmod.load_library()
    n_src, n, width = 1000, 3001, 4
    src = torch.from_numpy(gg.uniform_f32(n_src * width, 5)).cuda()
    idx_h = gg.uniform_int(n, n_src, 6).astype(np.int32)
    idx = torch.from_numpy(idx_h).cuda()
    dst = torch.full((n * width,), -1.0, device="cuda")
    vp = ctypes.c_void_p
    assert lib.tc_gather_rows(vp(src.data_ptr()), n_src, vp(idx.data_ptr()), n, width, vp(dst.data_ptr()), None) == 0
    want = src.cpu().numpy().reshape(n_src, width)[idx_h].ravel()
    assert np.array_equal(dst.cpu().numpy().view(np.uint32), want.view(np.uint32))
    # an index outside the source is an error, and nothing is written
    idx_h[n // 2] = n_src
    bad = torch.from_numpy(idx_h).cuda()
    dst.fill_(-1.0)
    assert lib.tc_gather_rows(vp(src.data_ptr()), n_src, vp(bad.data_ptr()), n, width, vp(dst.data_ptr()), None) != 0
    assert torch.all(dst == -1.0)


@pytest.mark.parametrize("scale,ef,every", [(10, 8, 7), (9, 12, 1), (11, 6, 30)])
def test_rwr_gradient_matches_fp64_reference(scale, ef, every):
    from test_oracle_rwr_grad import problem
    from oracle import rwr_grad as rg
    from paper_1103_2405_amd.rwr_grad import EdgeWeightedRWR
    n, rp, col, feats, theta, s, targets = problem(scale, ef, 31 + scale)
    model = EdgeWeightedRWR((n, n, rp, col), feats, s, 0.85, 30, every=every)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    r = model.scores(th)
    loss = -torch.log(r[torch.as_tensor(targets).cuda()].double()).sum()
    loss.backward()
    ref_loss, ref_grad, _ = rg.loss_and_grad(n, rp, col, feats, theta, s, targets, 0.85, 30)
    say("loss", loss.item(), ref_loss, "grad", th.grad.numpy(), ref_grad)
    assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss)
    assert np.linalg.norm(th.grad.numpy() - ref_grad) <= 1e-4 * np.linalg.norm(ref_grad)
    # the forward is the RWR driver's iteration on the same FP32 matrix
    one, _, _ = model.W.rwr([s], 0.85, 0.0, 30)
    assert torch.equal(one[:, 0], r.detach())
    model.close()


def test_rwr_gradient_does_not_depend_on_checkpoint_interval():
    from test_oracle_rwr_grad import problem
    from paper_1103_2405_amd.rwr_grad import EdgeWeightedRWR
    n, rp, col, feats, theta, s, targets = problem(9, 8, 77)
    grads = []
    for every in (1, 4, 30):
        model = EdgeWeightedRWR((n, n, rp, col), feats, s, 0.85, 30, every=every)
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        (-torch.log(model.scores(th)[torch.as_tensor(targets).cuda()].double()).sum()).backward()
        grads.append(th.grad.numpy().copy())
        model.close()
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[0], grads[2])


# ------------------------------------------------------------ TILE-COO
@pytest.mark.parametrize("W,split", [(64, -1), (512, 256), (1 << 20, 0)])
def test_tile_coo_format_and_products(W, split):
    g = gg.rmat(12, 16, seed=3)
    csr = gg.pagerank_matrix(g)
    gm, ref = build_both(csr, W, wl=1024, split_len=split, kernel="coo")
    fmt = gm.export_format()
    assert_same_format(fmt, ref)
    assert np.array_equal(fmt["coo_row"], ref["coo_row"]) and np.array_equal(fmt["coo_col"], ref["coo_col"])
    assert np.array_equal(fmt["coo_val"].view(np.uint32), ref["coo_val"].view(np.uint32))
    check_spmv(gm, csr, gg.uniform_f32(g.n, 9))


def test_tile_coo_dyadic_bit_exact_long_rows():
    # rows of 2500 entries cross several 512-entry intervals; every summation
    # order is exact on dyadic inputs, so the result must be bit-exact
    csr = _heavy_rows_csr(3000, 5, 2500, 6, 17, dyadic=True)
    rng = np.random.default_rng(3)
    x = rng.integers(-8, 9, size=csr[1]).astype(np.float32)
    for W in (1 << 20, 700):
        gm = TiledMatrix(csr, tile_width=W, kernel="coo")
        check_spmv(gm, csr, x, exact=True)
        assert gm.info()["kernel"] == 1


def test_tile_coo_pagerank_and_empty_rows():
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    gm = TiledMatrix(csr, tile_width=4096, kernel="coo")
    p, it, res = gm.pagerank(0.85, 0.0, 50)
    ref, _, _ = oracle.pagerank(csr, 0.85, 0.0, 50)
    assert np.abs(p.cpu().numpy() - ref).sum() <= 1e-6
    # the same iterates as the composite kernel to FP32 rounding
    pc, _, _ = TiledMatrix(csr, tile_width=4096).pagerank(0.85, 0.0, 50)
    assert np.abs(p.cpu().numpy() - pc.cpu().numpy()).sum() <= 1e-6


def test_dense_2000_matrix_both_kernels():
    # the paper's dense 2000 x 2000 sanity case (Section 4)
    n = 2000
    rp = np.arange(n + 1, dtype=np.int64) * n
    col = np.tile(np.arange(n, dtype=np.int32), n)
    val = gg.uniform_f32(n * n, 2000)
    csr = (n, n, rp, col, val)
    x = gg.uniform_f32(n, 2001)
    for kernel in ("composite", "coo"):
        check_spmv(TiledMatrix(csr, kernel=kernel), csr, x)


def test_rwr_gradient_of_an_earlier_forward():
    # two forwards on one model, then the backward of the first: the gradient
    # must be the first theta's (the model's state belongs to the second)
    from test_oracle_rwr_grad import problem
    from oracle import rwr_grad as rg
    from paper_1103_2405_amd.rwr_grad import EdgeWeightedRWR
    n, rp, col, feats, theta, s, targets = problem(9, 8, 78)
    model = EdgeWeightedRWR((n, n, rp, col), feats, s, 0.85, 30, every=7)
    tg = torch.as_tensor(targets).cuda()
    th1 = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    theta2 = np.asarray(theta) * -0.5 + 0.3
    th2 = torch.tensor(theta2, dtype=torch.float64, requires_grad=True)
    loss1 = -torch.log(model.scores(th1)[tg].double()).sum()
    loss2 = -torch.log(model.scores(th2)[tg].double()).sum()
    loss1.backward()
    loss2.backward()
    for th, t in ((th1, theta), (th2, theta2)):
        ref_loss, ref_grad, _ = rg.loss_and_grad(n, rp, col, feats, t, s, targets, 0.85, 30)
        say("grad", th.grad.numpy(), ref_grad)
        assert np.linalg.norm(th.grad.numpy() - ref_grad) <= 1e-4 * np.linalg.norm(ref_grad)
    model.close()


@pytest.mark.parametrize("W,split,wave", [(1 << 14, 256, 64), (2048, 128, 64), (1 << 14, 96, 32)])
def test_row_slices_do_not_change_results(W, split, wave):
    # the same format with 1, 2, 4 and 8 row slices forced on every tile:
    # column-major blocks, 64/128-wide and wider row-major rows, split-row
    # chunks and (wave 32) the generic path give bit-identical products and
    # PageRank iterates, within the bound of the oracle
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    x = torch.from_numpy(gg.uniform_f32(g.n, 101)).cuda()
    ys, ps = [], []
    for S in (1, 2, 4, 8):
        gm = TiledMatrix(csr, tile_width=W, split_len=split, wave=wave, slices=S)
        if S == 1:
            lay = gm.export_format(metadata_only=True)
            say("layouts", np.bincount(lay["wl_layout"], minlength=3), "w_pad", sorted(set(lay["wl_w_pad"].tolist()))[:8])
        ys.append(gm.spmv(x))
        ps.append(gm.pagerank(0.85, 0.0, 20)[0])
        gm.close()
    for S, y, p in zip((2, 4, 8), ys[1:], ps[1:]):
        assert torch.equal(y, ys[0]), S
        assert torch.equal(p, ps[0]), S
    xs = x.cpu().numpy()
    yy = ys[0].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(yy - oracle.spmv(csr, xs)) <= TOL * oracle.absmv(csr, xs))


@pytest.mark.parametrize("bounds,wl,split", [([300, 2000, 6000], 512, 256), ([16384], 2048, -1),
                                             ([64, 4096], 300, 64), ([1000, 1001, 9000, 16384], 1024, 128)])
def test_tiles_of_given_widths(bounds, wl, split):
    # tiles of different widths: the format bit for bit against the reference
    # builder, products within the bound, bit-exact on dyadic inputs, and
    # PageRank iterates against the oracle
    g = gg.rmat(14, 16, seed=14)
    csr = gg.pagerank_matrix(g)
    gm, ref = build_both(csr, W=4096, wl=wl, split_len=split, bounds=bounds)
    fmt = gm.export_format()
    assert_same_format(fmt, ref)
    check_spmv(gm, csr, gg.uniform_f32(g.n, 101))
    p, _, _ = gm.pagerank(0.85, 0.0, 30)
    pref, _, _ = oracle.pagerank(csr, 0.85, 0.0, 30)
    assert np.abs(p.cpu().numpy() - pref).sum() <= 1e-6
    gm.close()
    dy = gg.random_csr(3000, 3000, 0.004, 5, values="dyadic", power=1.2)
    x = ((np.arange(3000) * 7 + 5) % 7 - 3).astype(np.float32)
    gm2 = TiledMatrix(dy, wl=wl, split_len=split, tile_bounds=[b for b in bounds if b < 3000] or [3000])
    check_spmv(gm2, dy, x, exact=True)
    gm2.close()


def test_tile_bounds_rejected_when_invalid():
    csr = gg.pagerank_matrix(gg.rmat(9, 8, seed=2))
    for bad in ([0], [10, 10], [20, 10], [csr[1] + 1]):
        with pytest.raises(TcError):
            TiledMatrix(csr, tile_bounds=bad)


@pytest.mark.parametrize("bounds,wl,split,S", [([4096], 512, 128, 0), ([32768], 1024, 256, 4), ([333, 9000], 300, 64, 2),
                                               ([1024, 2048, 3072], 2048, -1, 1)])
def test_lds_staged_tiles(bounds, wl, split, S):
    # tiles whose x segment is staged in LDS (forced on every tile that fits):
    # the same format as without staging, the products bit-identical to the
    # cache-gather kernel's, within the oracle's bound and bit-exact on
    # dyadic inputs; PageRank iterates against the oracle
    g = gg.rmat(15, 16, seed=15)
    csr = gg.pagerank_matrix(g)
    x = torch.from_numpy(gg.uniform_f32(g.n, 101)).cuda()
    a = TiledMatrix(csr, wl=wl, split_len=split, tile_bounds=bounds, lds_stage=1, slices=S)
    b = TiledMatrix(csr, wl=wl, split_len=split, tile_bounds=bounds, lds_stage=-1, slices=S)
    ya, yb = a.spmv(x), b.spmv(x)
    assert torch.equal(ya, yb)
    xs = x.cpu().numpy()
    assert np.all(np.abs(ya.cpu().numpy().astype(np.float64) - oracle.spmv(csr, xs)) <= TOL * oracle.absmv(csr, xs))
    pa = a.pagerank(0.85, 0.0, 25)[0]
    assert torch.equal(pa, b.pagerank(0.85, 0.0, 25)[0])
    pref, _, _ = oracle.pagerank(csr, 0.85, 0.0, 25)
    assert np.abs(pa.cpu().numpy() - pref).sum() <= 1e-6
    a.close()
    b.close()
    dy = gg.random_csr(50000, 50000, 0.0004, 6, values="dyadic", power=1.3)
    xd = ((np.arange(50000) * 7 + 6) % 7 - 3).astype(np.float32)
    gm = TiledMatrix(dy, wl=wl, split_len=split, tile_bounds=bounds, lds_stage=1, slices=S)
    check_spmv(gm, dy, xd, exact=True)
    gm.close()


# ------------------------------------------------------------ measurement kernels
def test_stream_and_gather_read_measurement_kernels():
    # the attainable-rate kernels of the roofline read every element once:
    # their per-thread sums add up to the exact totals (small integers)
    from paper_1103_2405_amd.tc import STREAM_SINK_FLOATS, gather_read, stream_read
    sink = torch.zeros(STREAM_SINK_FLOATS, device="cuda")
    a = torch.ones(1 << 22, device="cuda")
    stream_read(a, sink)
    assert sink.double().sum().item() == float(1 << 22)
    n = 1 << 20
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    x = torch.ones(1000, device="cuda")
    x[0] = 2.0
    idx = torch.randint(1, 1000, (n,), device="cuda", dtype=torch.int32, generator=gen)
    idx[:3] = torch.tensor([-1, 1000, 1 << 30], dtype=torch.int32)  # outside [0, n_x): x[0]
    val = torch.ones(n, device="cuda")
    sink.zero_()
    gather_read(x, idx, val, sink)
    assert sink.double().sum().item() == float(n + 3)
    with pytest.raises(TcError):
        gather_read(x, idx[:1000], val[:1000], sink)  # not a multiple of 512
