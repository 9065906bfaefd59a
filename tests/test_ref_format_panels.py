"""Row panels in the reference builder (CPU): the panel bounds rule worked by
hand, the per-row weights against a brute-force count, the format's round
trip and product, and the reduction to the plain format with one panel.

Row panels are the row partition of Section 3.2 (rows of a large matrix split
into blocks, each block tiled and tuned on its own) applied to the workgroups
of one GPU: every (panel, column tile) pair is a tile of the format.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import ref_format as rf
from oracle.autotune import tile_split_len


def test_panel_bounds_hand_worked():
    # weights 5 1 1 1 4 0 3 (total 15), 3 panels of at most 3 rows:
    # prefix 0 5 6 7 8 12 12 15; targets 5, 10, 15 -> lower bounds 1, 5, 7;
    # panel 1 is cut at 1 + 3 = 4 rows by the row cap, panel 2 ends at 7
    assert rf.panel_bounds(np.array([5, 1, 1, 1, 4, 0, 3]), 3, 3) == [0, 1, 4, 7]
    # no weight: every panel takes one row, the rest go into panels of max_rows
    assert rf.panel_bounds(np.zeros(5, np.int64), 2, 2) == [0, 1, 2, 4, 5]
    # more panels than rows: one row each, then stop
    assert rf.panel_bounds(np.array([1, 1]), 5, 10) == [0, 1, 2]
    assert rf.panel_bounds(np.zeros(0, np.int64), 4, 8) == [0]
    with pytest.raises(ValueError):
        rf.panel_bounds(np.ones(3, np.int64), 1, 0)


def test_panel_bounds_properties():
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = int(rng.integers(1, 400))
        w = rng.integers(0, 30, n) * (rng.random(n) < 0.8)
        P, R = int(rng.integers(1, 40)), int(rng.integers(1, 60))
        b = rf.panel_bounds(w, P, R)
        d = np.diff(b)
        assert b[0] == 0 and b[-1] == n and (d >= 1).all() and (d <= R).all()
        pre = np.concatenate([[0], np.cumsum(w)])
        tot = pre[-1]
        for p in range(min(P, len(b) - 1)):
            tgt = -(-((p + 1) * tot) // P)
            # panel p ends at the first row reaching its target, unless a cap bites
            lb = int(np.searchsorted(pre, tgt, side="left"))
            assert b[p + 1] == min(max(lb, b[p] + 1), b[p] + R, n)


def test_panel_weights_brute_force():
    csr = gg.random_csr(120, 120, 0.08, 11, power=1.2)
    n, _, rp, col, _ = csr
    ctile = np.minimum(col // 16, 5)
    irow = np.repeat(np.arange(n), np.diff(rp))
    split = [3, 0, 2, 5, 1, 4]
    w = rf.panel_weights(n, irow, ctile, split)
    for r in range(n):
        exp = 0
        for t in range(6):
            L = int(np.sum(ctile[rp[r]:rp[r + 1]] == t))
            if split[t] == 0 or L <= split[t]:
                exp += L
        assert w[r] == exp


@pytest.mark.parametrize("seed,n_rows,n_cols,W,split,P,R", [
    (0, 300, 300, 16, 0, 7, 64),
    (1, 500, 500, 40, 6, 16, 40),
    (2, 250, 700, 50, -1, 5, 80),   # rectangular: original row ids
    (3, 400, 400, 400, 3, 33, 16),  # one column tile
])
def test_panel_format_round_trip_and_product(seed, n_rows, n_cols, W, split, P, R):
    csr = gg.random_csr(n_rows, n_cols, 0.03, seed, power=1.1)
    f = rf.build(csr, W=W, wl=[37] * 100000, S=4, split_len=split, panels=P, panel_rows=R, panel_waves=4)
    NT, pb = f["n_col_tiles"], f["panel_begin"]
    assert f["n_tiles_total"] == (len(pb) - 1) * NT
    assert pb[0] == 0 and pb[-1] == n_rows and (np.diff(pb) <= R).all()
    # every tile's rows lie in its panel; its pads and entries in its column tile
    for g in range(f["n_tiles_total"]):
        rows = f["rows_sorted"][f["tile_row_off"][g]:f["tile_row_off"][g + 1]]
        p = g // NT
        assert ((rows >= pb[p]) & (rows < pb[p + 1])).all()
        assert f["tile_col_begin"][g] == f["tile_col_begin"][g % NT] and f["tile_split"][g] == f["tile_split"][g % NT]
    sel = f["wl_tile"]
    for j in range(len(sel)):
        g = int(sel[j])
        seg = f["idx"][f["wl_data_off"][j]:f["wl_data_off"][j] + f["wl_w_pad"][j] * f["wl_h_pad"][j]]
        assert ((seg >= f["tile_col_begin"][g]) & (seg < max(f["tile_col_end"][g], f["tile_col_begin"][g] + 1))).all()
    # round trip and product
    r, c, v = rf.decode_coo(f)
    n, m, rp, col, val = csr
    r0 = np.repeat(np.arange(n), np.diff(rp))
    o = np.lexsort((val.view(np.uint32), col, r0))
    assert np.array_equal(r, r0[o]) and np.array_equal(c, col[o]) and np.array_equal(v.view(np.uint32), val[o].view(np.uint32))
    x = gg.uniform_f32(m, 5)
    dense = np.zeros((n, m))
    np.add.at(dense, (r0, col), val.astype(np.float64))
    assert np.allclose(rf.spmv_format(f, x), dense @ x.astype(np.float64), rtol=1e-12, atol=1e-12)


def test_one_panel_is_the_plain_format():
    # one panel holding every row: tile g = column tile g, so with given
    # workload sizes every array equals the format built without panels
    csr = gg.random_csr(400, 400, 0.02, 9, power=1.2)
    a = rf.build(csr, W=48, wl=[50] * 100, S=8, split_len=5)
    b = rf.build(csr, W=48, wl=[50] * 100, S=8, split_len=5, panels=1, panel_rows=400)
    for k in ("tile_col_begin", "tile_col_end", "tile_nnz", "tile_split", "tile_row_off", "rows_sorted", "rows_len",
              "wl_tile", "wl_layout", "wl_w_pad", "wl_h_pad", "wl_row_begin", "wl_data_off", "wl_rowid_off", "idx",
              "rowid"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    assert np.array_equal(a["val"].view(np.uint32), b["val"].view(np.uint32))


def test_panel_split_length_is_the_column_tiles():
    # chunking follows the column tile's entries, not the (panel, tile)'s
    csr = gg.random_csr(300, 300, 0.05, 2, power=1.3)
    f = rf.build(csr, W=30, wl=[64] * 10000, S=4, split_len=-1, max_act_warp=64, panels=6, panel_rows=60)
    NT = f["n_col_tiles"]
    for t in range(NT):
        nnz_t = int(sum(f["tile_nnz"][g] for g in range(t, f["n_tiles_total"], NT)))
        assert f["tile_split"][t] == tile_split_len(-1, nnz_t, 64, 4)
