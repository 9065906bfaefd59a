"""Row panels on the GPU, through the C ABI: the format bit for bit against
the reference builder (given and autotuned workload sizes), the one-launch
panel pass bit-identical to one launch per tile, products within the per-entry
bound of the oracle (bit-exact on dyadic inputs), the same bits for every
workgroup size, and PageRank iterates against the oracle.

Row panels are the row partition of Section 3.2 applied to the workgroups of
one GPU: each (panel, column tile) pair is a tile of the format."""
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

from paper_1103_2405_amd import TcError, TiledMatrix  # noqa: E402

TOL = 1e-5
FMT_KEYS = ["cperm", "rowmap", "tile_col_begin", "tile_col_end", "tile_nnz", "tile_wl", "tile_split", "tile_row_off",
            "rows_sorted", "rows_len", "wl_tile", "wl_layout", "wl_w", "wl_w_pad", "wl_h_pad", "wl_row_begin",
            "wl_n_rows", "wl_chunk", "wl_n_chunks", "wl_data_off", "wl_rowid_off", "idx", "rowid", "panel_begin"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same_format(g, r):
    assert g["T"] == r["T"] and g["n_tiles_total"] == r["n_tiles_total"] and g["nnz_pad"] == r["nnz_pad"]
    assert g["n_col_tiles"] == r["n_col_tiles"]
    for k in FMT_KEYS:
        a, b = np.asarray(g[k]), np.asarray(r[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), k
    assert np.array_equal(g["val"].view(np.uint32), r["val"].view(np.uint32)), "val"


def build_pair(csr, W, P, R, waves=16, wl=None, split=-1, S=64, table=None, max_act_warp=8192, bounds=None):
    say("panels build", csr[0], csr[1], len(csr[3]), "W", W, "P", P, "R", R, "waves", waves, "wl", wl, "split", split)
    gm = TiledMatrix(csr, tile_width=W, wl=wl, wave=S, split_len=split, perf_table=table, max_act_warp=max_act_warp,
                     panels=P, panel_rows=R, panel_waves=waves, tile_bounds=bounds)
    ref = rf.build(csr, W=W, wl=None if wl is None else [wl] * 1000000, S=S, split_len=split,
                   table=PerfTable.load(table) if table else None, max_act_warp=max_act_warp, bounds=bounds,
                   panels=P, panel_rows=R, panel_waves=waves)
    return gm, ref


def check_products(gm, csr, x, exact=False):
    xt = torch.from_numpy(x).cuda()
    ya = torch.empty(csr[0], device="cuda")
    yb = torch.empty(csr[0], device="cuda")
    gm.spmv_internal(xt, ya)  # internal ids: the two passes are compared bit for bit
    gm.spmv_tiles(xt, yb)
    assert torch.equal(ya.view(torch.int32), yb.view(torch.int32)), "panel pass differs from the tile-by-tile pass"
    y = gm.spmv(xt).cpu().numpy().astype(np.float64)
    ref = oracle.spmv(csr, x)
    if exact:
        assert np.array_equal(y, ref)
        return
    err = np.abs(y - ref)
    bound = TOL * oracle.absmv(csr, x)
    bad = np.flatnonzero(err > bound)
    assert bad.size == 0, (bad[:10], err[bad[:10]], bound[bad[:10]])


@pytest.mark.parametrize("seed,n,density,W,wl,split,P,R", [
    (0, 600, 0.02, 64, 128, 0, 7, 128),
    (1, 2000, 0.006, 256, 300, 40, 16, 200),
    (2, 3000, 0.004, 3000, 512, -1, 5, 1024),
    (3, 1500, 0.01, 100, 64, 16, 40, 64),
])
def test_panel_format_bit_exact_and_products(seed, n, density, W, wl, split, P, R):
    csr = gg.random_csr(n, n, density, seed, power=1.2)
    gm, ref = build_pair(csr, W, P, R, wl=wl, split=split)
    f = gm.export_format()
    assert f["n_panels"] == len(ref["panel_begin"]) - 1
    same_format(f, ref)
    check_products(gm, csr, gg.uniform_f32(n, seed + 50))


def test_panel_format_rectangular():
    csr = gg.random_csr(900, 400, 0.01, 4, power=1.0)
    gm, ref = build_pair(csr, 100, 9, 150, wl=200, split=24)
    same_format(gm.export_format(), ref)
    check_products(gm, csr, gg.uniform_f32(400, 3))


def test_panel_autotuned_sizes_match_reference(tmp_path):
    from test_gpu_parity import _write_table
    path = str(tmp_path / "table.txt")
    _write_table(path)
    csr = gg.pagerank_matrix(gg.rmat(13, 16, seed=3))
    for waves in (4, 16):
        gm, ref = build_pair(csr, 1024, 12, 1024, waves=waves, table=path, max_act_warp=256)
        f = gm.export_format()
        assert list(f["tile_wl"]) == list(ref["tile_wl"]) and len(set(ref["tile_wl"])) > 1
        same_format(f, ref)
        check_products(gm, csr, gg.uniform_f32(csr[0], 5))


def test_panel_given_bounds_and_rmat14():
    csr = gg.pagerank_matrix(gg.rmat(14, 16, seed=14))
    gm, ref = build_pair(csr, 1 << 14, 64, 512, wl=1024, split=512, bounds=[512, 2048, 8192])
    same_format(gm.export_format(), ref)
    check_products(gm, csr, gg.uniform_f32(csr[0], 101))


@pytest.mark.parametrize("seed", [0, 1])
def test_panel_dyadic_bit_exact(seed):
    csr = gg.random_csr(3000, 3000, 0.004, seed, values="dyadic", power=1.2)
    x = ((np.arange(3000) * 7 + seed) % 7 - 3).astype(np.float32)
    gm = TiledMatrix(csr, tile_width=256, wl=300, split_len=16, panels=24, panel_rows=256)
    check_products(gm, csr, x, exact=True)


def test_panel_waves_give_the_same_bits():
    csr = gg.pagerank_matrix(gg.rmat(13, 16, seed=8))
    x = torch.from_numpy(gg.uniform_f32(csr[0], 9)).cuda()
    ys = []
    for waves in (4, 8, 16):
        gm = TiledMatrix(csr, tile_width=1024, wl=512, split_len=256, panels=20, panel_rows=1024, panel_waves=waves)
        y = torch.empty(csr[0], device="cuda")
        gm.spmv_internal(x, y)
        ys.append(y.view(torch.int32).cpu())
    assert torch.equal(ys[0], ys[1]) and torch.equal(ys[0], ys[2])


def reference_of(gm, csr, table, P):
    """The reference builder with the panel count asked for and the parameters
    a handle reports (automatic panels: head tile, column tiles, panel size)."""
    inf = gm.info()
    f = gm.export_format(metadata_only=True)
    T = inf["n_dense_tiles"]
    # automatic panels: workloads of 512 entries, rows split beyond 1024
    return rf.build(csr, W=inf["tile_width"], bounds=[int(v) for v in f["tile_col_end"][:T]],
                    wl=[512] * inf["n_tiles"], split_len=1024, panels=P, panel_rows=inf["panel_rows"],
                    panel_waves=inf["panel_waves"])


@pytest.mark.parametrize("scale", [12, 14])
def test_panel_automatic_format_and_pagerank(scale):
    from paper_1103_2405_amd.tc import DEFAULT_PERF_TABLE
    csr = gg.pagerank_matrix(gg.rmat(scale, 16, seed=scale))
    gm = TiledMatrix(csr, panels=-1, tile_width=1024)
    inf = gm.info()
    say(inf)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    P = min(n_cu, -(-csr[0] // 2048))
    R = ((17 * (-(-csr[0] // P)) + 15) // 16 + 63) // 64 * 64
    # P panels are asked for; the row cap can leave rows for further panels
    assert inf["n_panels"] >= P and inf["panel_rows"] == max(64, R) and inf["panel_waves"] == 16
    assert inf["split_len"] == 1024 and set(gm.export_format(metadata_only=True)["tile_wl"]) == {512}
    assert (np.diff(gm.export_format(metadata_only=True)["panel_begin"]) <= inf["panel_rows"]).all()
    f = gm.export_format()
    head = f["tile_col_end"][0]
    assert head % 1024 == 0 or head == csr[1]
    same_format(f, reference_of(gm, csr, DEFAULT_PERF_TABLE, P))
    check_products(gm, csr, gg.uniform_f32(csr[0], 3))
    p, it, res = gm.pagerank(0.85, 0.0, 50)
    pref, _, _ = oracle.pagerank(csr, 0.85, 0.0, 50)
    assert np.abs(p.cpu().numpy().astype(np.float64) - pref).sum() <= 1e-6


def test_panel_edge_cases():
    # empty matrix, one row, more panels than rows
    z = (0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    gm = TiledMatrix(z, panels=4, panel_rows=16)
    assert gm.info()["n_panels"] == 0
    one = (1, 1, np.array([0, 1], np.int64), np.zeros(1, np.int32), np.ones(1, np.float32))
    gm = TiledMatrix(one, panels=3, panel_rows=8)
    check_products(gm, one, np.array([2.0], np.float32), exact=True)
    csr = gg.random_csr(50, 50, 0.1, 1)
    gm = TiledMatrix(csr, tile_width=16, wl=32, panels=200, panel_rows=4)
    assert gm.info()["n_panels"] == 50
    check_products(gm, csr, gg.uniform_f32(50, 2))


def test_panel_invalid_options():
    csr = gg.random_csr(100, 100, 0.05, 1)
    for kw in (dict(panels=4, xcd_groups=2), dict(panels=4, kernel="coo"), dict(panels=-2), dict(panels=4, panel_waves=3),
               dict(panels=4, panel_rows=1 << 20)):
        with pytest.raises(TcError):
            TiledMatrix(csr, **kw)


@pytest.mark.parametrize("bounds,R", [([64, 600, 1800], 700), ([1000], 2000), ([3, 50], 300)])
def test_panel_lds_staged_first_tile(bounds, R):
    """A narrow first column tile is staged in LDS behind the panel's y: the
    format is the reference's, and the products are the tile-by-tile bits."""
    csr = gg.random_csr(2500, 2500, 0.006, 12, power=1.3)
    gm, ref = build_pair(csr, 2500, 9, R, wl=256, split=32, bounds=bounds)
    same_format(gm.export_format(), ref)
    check_products(gm, csr, gg.uniform_f32(2500, 13))
    off = TiledMatrix(csr, wl=256, split_len=32, tile_bounds=bounds, panels=9, panel_rows=R, lds_stage=-1)
    x = torch.from_numpy(gg.uniform_f32(2500, 14)).cuda()
    ya, yb = torch.empty(2500, device="cuda"), torch.empty(2500, device="cuda")
    gm.spmv_internal(x, ya)
    off.spmv_internal(x, yb)
    assert torch.equal(ya.view(torch.int32), yb.view(torch.int32))


@pytest.mark.parametrize("split,bounds", [(-1, None), (64, [512, 2048]), (16, [1024])])
def test_panel_pagerank_fused_update_equals_separate_update(split, bounds):
    """With the change read every iteration no step is fused; with a fixed
    count every step but the last runs the update inside the panel pass: the
    iterates agree bit for bit (split rows with and without unsplit segments,
    rows without entries and dangling columns included)."""
    csr = gg.pagerank_matrix(gg.rmat(13, 8, seed=21))
    assert np.any(np.diff(csr[2]) == 0) and np.any(np.bincount(csr[3], minlength=csr[1]) == 0)
    gm = TiledMatrix(csr, tile_width=1024, split_len=split, tile_bounds=bounds, panels=11, panel_rows=1024)
    inf = gm.info()
    assert inf["n_panels"] >= 11 and (split < 0 or inf["n_split_rows"] > 0)
    a, it, ra = gm.pagerank(0.85, 1e-7, 300, check_every=1)
    b, it2, rb = gm.pagerank(0.85, 0.0, it)
    assert it2 == it and ra == rb
    assert torch.equal(a, b)
    pref, _, _ = oracle.pagerank(csr, 0.85, 0.0, it)
    assert np.abs(b.cpu().numpy() - pref).sum() <= 1e-6


def test_panel_hits_and_rwr_match_oracle():
    # the HITS and RWR drivers on row-panel handles: single vectors through
    # the panel pass, several RWR queries through the tile-by-tile SpMM
    g = gg.rmat(13, 16, seed=9)
    csr = gg.hits_matrix(g)
    tm = TiledMatrix(csr, panels=-1)
    assert tm.info()["n_panels"] > 1
    a, h, it, _ = tm.hits(0.0, 30)
    x, _, _ = oracle.hits(csr, 0.0, 30)
    n = g.n
    d = np.abs(a.cpu().numpy() - x[:n]).sum() + np.abs(h.cpu().numpy() - x[n:]).sum()
    say("panel hits L1 diff", d)
    assert it == 30 and d <= 1e-6
    tm.close()
    csr = gg.rwr_matrix(g)
    tm = TiledMatrix(csr, panels=-1)
    seeds = gg.rwr_seeds(g, 8, 9)
    for k in (1, 5):
        R, it, _ = tm.rwr(seeds[:k], 0.85, 0.0, 30)
        Rref, _, _ = oracle.rwr(csr, seeds[:k], 0.85, 0.0, 30)
        d = np.abs(R.cpu().numpy().reshape(Rref.shape) - Rref).sum(axis=0)
        say("panel rwr k", k, "L1 diff per column", d)
        assert np.all(d <= 1e-6)
    tm.close()
