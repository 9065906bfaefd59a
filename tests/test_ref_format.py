"""Pins of the reference format builder: the paper's worked example
(Figure 1, described in Section 3.1), structural invariants, an exact round
trip back to the input entries, and special cases whose format is known."""
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import ref_format as rf
from oracle.autotune import RM, CM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_fig1():
    entries, params, expect = [], {}, []
    with open(os.path.join(GOLDEN, "fig1_example.txt")) as f:
        mode = None
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line == "entries":
                mode = "e"
                continue
            if line == "end":
                mode = None
                continue
            if mode == "e":
                r, c, v = line.split()
                entries.append((int(r), int(c), float(v)))
            elif line.startswith("tile0"):
                _, lay, w, h = line.split()
                expect.append((lay, int(w), int(h)))
            else:
                k, v = line.split()
                params[k] = int(v)
    n = 1 + max(max(e[0], e[1]) for e in entries)
    entries.sort()
    rp = np.zeros(n + 1, np.int64)
    for r, _, _ in entries:
        rp[r + 1] += 1
    rp = np.cumsum(rp)
    col = np.array([e[1] for e in entries], np.int32)
    val = np.array([e[2] for e in entries], np.float32)
    return (n, n, rp, col, val), params, expect


def test_figure1_worked_example():
    csr, p, expect = load_fig1()
    fmt = rf.build(csr, W=p["W"], wl=[p["WL"]] * 3, S=p["S"], split_len=0)
    assert fmt["T"] == p["T"]
    t0 = fmt["wl_tile"] == 0
    got = [("RM" if fmt["wl_layout"][j] == RM else "CM",
            int(fmt["wl_w_pad"][j]) if fmt["wl_layout"][j] == RM else int(fmt["wl_w"][j]),
            int(fmt["wl_n_rows"][j])) for j in np.flatnonzero(t0)]
    assert got == expect
    # tile 0 holds the two longest columns (each of length 6), sorted rows 2,2,2,2,1,1,1,1
    assert list(fmt["clen"][fmt["cperm"][:2]]) == [6, 6]
    assert list(fmt["rows_len"][fmt["tile_row_off"][0]:fmt["tile_row_off"][1]]) == [2, 2, 2, 2, 1, 1, 1, 1]
    check_invariants(csr, fmt)


def check_invariants(csr, fmt):
    n_rows, n_cols, rp, col, val = csr
    S = fmt["S"]
    cperm = fmt["cperm"].astype(np.int64)
    assert np.array_equal(np.sort(cperm), np.arange(n_cols))
    clen = np.bincount(col, minlength=n_cols)
    cs = clen[cperm]
    assert np.all(np.diff(cs) <= 0)
    same = np.diff(cs) == 0
    assert np.all(np.diff(cperm)[same] > 0)  # ties by ascending id
    # tiles: contiguous, cover all columns, dense ones W wide
    b, e = fmt["tile_col_begin"], fmt["tile_col_end"]
    if len(b):
        assert b[0] == 0 and e[-1] == n_cols and np.all(b[1:] == e[:-1])
    if not fmt.get("xcd_groups") and not fmt.get("bounds"):
        for t in range(fmt["T"]):
            assert b[t] == t * fmt["W"]
            assert cs[b[t]] >= 2 or fmt["T"] == 0
    # per-tile rows sorted by decreasing length, ties by increasing row id
    for t in range(fmt["n_tiles_total"]):
        L = fmt["rows_len"][fmt["tile_row_off"][t]:fmt["tile_row_off"][t + 1]]
        Rr = fmt["rows_sorted"][fmt["tile_row_off"][t]:fmt["tile_row_off"][t + 1]]
        assert np.all(np.diff(L) <= 0) and np.all(L > 0)
        assert np.all(np.diff(Rr)[np.diff(L) == 0] > 0)
    # workloads: padding multiple of S on the padded side, offsets increasing
    for j in range(len(fmt["wl_tile"])):
        lay, wp, hp = fmt["wl_layout"][j], fmt["wl_w_pad"][j], fmt["wl_h_pad"][j]
        if lay == RM:
            # a multiple of S, or S / 2 for rows of at most half of S = 64
            half = S >= 64 and wp == S // 2 and fmt["wl_w"][j] <= S // 2
            assert (wp % S == 0 or half) and wp >= fmt["wl_w"][j]
        else:
            assert hp % S == 0 and fmt["wl_w"][j] < hp
        if j + 1 < len(fmt["wl_tile"]):
            assert fmt["wl_data_off"][j + 1] >= fmt["wl_data_off"][j] + wp * hp
    # round trip: exactly the input entries
    r, c, v = rf.decode_coo(fmt)
    rows = np.repeat(np.arange(n_rows), np.diff(rp))
    o = np.lexsort((val.view(np.uint32), col, rows))
    assert np.array_equal(r, rows[o]) and np.array_equal(c, col[o].astype(np.int64))
    assert np.array_equal(v.view(np.uint32), val[o].view(np.uint32))
    # pads: value +0.0 and a valid column
    real = np.zeros(fmt["nnz_pad"], bool)
    for j in range(len(fmt["wl_tile"])):
        rb, nr, off = fmt["wl_row_begin"][j], fmt["wl_n_rows"][j], fmt["wl_data_off"][j]
        wp, hp, lay = fmt["wl_w_pad"][j], fmt["wl_h_pad"][j], fmt["wl_layout"][j]
        if fmt["wl_chunk"][j] >= 0:
            real[off:off + fmt["wl_w"][j]] = True
            continue
        for q in range(nr):
            L = fmt["rows_len"][rb + q]
            cs_ = np.arange(L)
            real[off + (q * wp + cs_ if lay == RM else cs_ * hp + q)] = True
    assert np.all(fmt["val"][~real].view(np.uint32) == 0)
    tb = fmt["tile_col_begin"][fmt["wl_tile"]] if len(fmt["wl_tile"]) else np.zeros(0)
    assert real.sum() == len(col)
    assert np.all((fmt["idx"] >= 0) & (fmt["idx"] < max(n_cols, 1)))
    # each stored column falls in its workload's tile
    for j in range(len(fmt["wl_tile"])):
        t = fmt["wl_tile"][j]
        off = fmt["wl_data_off"][j]
        seg = fmt["idx"][off:off + fmt["wl_w_pad"][j] * fmt["wl_h_pad"][j]]
        assert np.all((seg >= b[t]) & (seg < e[t]))


@pytest.mark.parametrize("seed,W,wl,S,split", [(0, 16, 64, 64, 0), (1, 7, 12, 4, 0), (2, 32, 200, 64, 40),
                                               (3, 5, 3, 2, 6), (4, 1000, 500, 64, 100)])
def test_invariants_and_round_trip(seed, W, wl, S, split):
    csr = gg.random_csr(300, 300, 0.03, seed, power=1.1)
    fmt = rf.build(csr, W=W, wl=[wl] * 400, S=S, split_len=split)
    check_invariants(csr, fmt)
    x = gg.uniform_f32(300, seed)
    assert np.allclose(rf.spmv_format(fmt, x), oracle.spmv(csr, x), rtol=1e-12, atol=1e-14)


def test_rectangular_matrix_keeps_row_ids():
    csr = gg.random_csr(90, 250, 0.05, 5, power=1.0)
    fmt = rf.build(csr, W=20, wl=[30] * 100, S=8, split_len=0)
    assert not fmt["relabel"] and np.array_equal(fmt["rowmap"], np.arange(90))
    check_invariants(csr, fmt)


def test_all_columns_short_gives_sparse_tile_only():
    n = 50
    rp = np.arange(n + 1, dtype=np.int64)
    col = np.random.default_rng(0).permutation(n).astype(np.int32)
    csr = (n, n, rp, col, np.ones(n, np.float32))
    fmt = rf.build(csr, W=8, wl=[64], S=64, split_len=0)
    assert fmt["T"] == 0 and fmt["n_tiles_total"] == 1
    check_invariants(csr, fmt)


def test_diagonal_is_one_column_major_column():
    n = 100
    csr = (n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n, np.float32))
    fmt = rf.build(csr, W=64, wl=[1 << 20], S=64, split_len=0)
    assert fmt["T"] == 0
    assert list(fmt["wl_layout"]) == [CM] and fmt["wl_w"][0] == 1 and fmt["wl_h_pad"][0] == 128
    assert fmt["wl_n_rows"][0] == 100
    check_invariants(csr, fmt)


def test_dense_matrix_workloads_identical():
    n = 128
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    csr = (n, n, rp, col, np.ones(n * n, np.float32))
    fmt = rf.build(csr, W=n, wl=[n * 4], S=64, split_len=0)
    assert fmt["T"] == 1 and fmt["n_tiles_total"] == 1
    assert set(zip(fmt["wl_layout"], fmt["wl_w_pad"], fmt["wl_h_pad"])) == {(RM, 128, 4)}
    assert fmt["nnz_pad"] == n * n
    check_invariants(csr, fmt)


def test_wl_equal_first_row_gives_one_row_per_workload():
    csr = gg.random_csr(64, 64, 0.5, 2)
    fmt = rf.build(csr, W=64, n_tiles=1, wl=[1], S=4, split_len=0)
    L0 = fmt["rows_len"][0]
    fmt = rf.build(csr, W=64, n_tiles=1, wl=[int(L0)], S=4, split_len=0)
    assert fmt["wl_n_rows"][0] == 1 and fmt["wl_layout"][0] == RM
    check_invariants(csr, fmt)


def test_split_heavy_rows_into_chunks():
    n = 40
    rows = np.concatenate([np.zeros(35, int), np.full(10, 3), np.arange(n)])
    cols = np.concatenate([np.arange(35), np.arange(10), (np.arange(n) * 7) % n])
    key = np.unique(rows * n + cols)
    r, c = key // n, (key % n).astype(np.int32)
    rp = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))]).astype(np.int64)
    csr = (n, n, rp, c, gg.uniform_f32(len(c), 3))
    fmt = rf.build(csr, W=1000, wl=[16], S=4, split_len=8)
    ch = fmt["wl_chunk"] >= 0
    assert ch.sum() >= 5 and np.all(fmt["wl_n_rows"][ch] == 1) and np.all(fmt["wl_h_pad"][ch] == 1)
    check_invariants(csr, fmt)
    x = gg.uniform_f32(n, 4)
    assert np.allclose(rf.spmv_format(fmt, x), oracle.spmv(csr, x), rtol=1e-12)


def test_partition_camping_pad():
    n = 64
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    csr = (n, n, rp, col, np.ones(n * n, np.float32))
    fmt = rf.build(csr, W=n, wl=[n * 8], S=64, split_len=0, camping_pad=True)
    # every workload is 64 x 8 = 512 floats, so 64 pad floats follow each one
    assert np.all(np.diff(fmt["wl_data_off"]) == 512 + 64)
    check_invariants(csr, fmt)


@pytest.mark.parametrize("seed,W,groups", [(0, 16, 8), (1, 1, 4), (2, 500, 8), (3, 40, 3)])
def test_xcd_column_ranges(seed, W, groups):
    """Head tile [0, W) then `groups` column ranges of (nearly) equal entries:
    every range's entry count is within one column length of rest / groups."""
    csr = gg.random_csr(400, 400, 0.02, seed, power=1.2)
    fmt = rf.build(csr, W=W, wl=[64] * 20, S=64, split_len=-1, xcd_groups=groups)
    check_invariants(csr, fmt)
    b, e, nz = fmt["tile_col_begin"], fmt["tile_col_end"], fmt["tile_nnz"]
    assert len(b) == groups + 1 and b[0] == 0 and e[0] == min(W, 400)
    cs = fmt["clen"][fmt["cperm"].astype(np.int64)]
    rest = int(cs[e[0]:].sum())
    for g in range(1, groups + 1):
        # prefix of the rest at the end of range g reaches ceil(g * rest / groups) at the first column
        pre_end = int(cs[e[0]:e[g]].sum())
        assert pre_end >= min(rest, -(-(g * rest) // groups)) or e[g] == 400
        if e[g] > e[0]:
            assert int(cs[e[0]:e[g] - 1].sum()) < -(-(g * rest) // groups) or g == groups
    x = gg.uniform_f32(400, seed)
    assert np.allclose(rf.spmv_format(fmt, x), oracle.spmv(csr, x), rtol=1e-12, atol=1e-14)


def test_coo_arrays_follow_the_bucketed_order():
    # the coordinate arrays of TILE-COO: every entry once, tiles ascending,
    # rows ascending in a tile, and the add flag exactly on rows an earlier
    # tile already holds
    csr = gg.random_csr(40, 50, 0.2, 3, power=1.2)
    f = rf.build(csr, W=8, wl=[64] * 100, S=4, coo=True)
    assert len(f["coo_row"]) == f["nnz"]
    flag = (f["coo_row"] >> 30) & 1
    row = f["coo_row"] & ((1 << 30) - 1)
    tile = np.repeat(np.arange(f["n_tiles_total"]), f["tile_nnz"])
    assert np.all(np.diff(tile * (1 << 31) + row.astype(np.int64)) >= 0)
    seen = set()
    for t, r, fl in zip(tile, row, flag):
        assert fl == (1 if any(s[1] == r and s[0] < t for s in seen) else 0)
        seen.add((t, r))
    # same multiset of (internal row, internal column, value) as the matrix
    n, _, rp, col, val = csr
    rows = np.repeat(np.arange(n), np.diff(rp))
    want = sorted(zip(f["rowmap"][rows].tolist(), f["cpos"][col].tolist(), val.view(np.uint32).tolist()))
    got = sorted(zip(row.tolist(), f["coo_col"].tolist(), f["coo_val"].view(np.uint32).tolist()))
    assert want == got


@pytest.mark.parametrize("seed,bounds,wl,split", [(0, [5, 37, 120], 64, 0), (1, [300], 40, 16),
                                                  (2, [1, 2, 3, 250], 30, -1), (3, [64, 128], 200, 32)])
def test_tiles_of_given_widths(seed, bounds, wl, split):
    # tiles of different widths (one per cache level): the invariants, the
    # exact round trip, and each tile's columns exactly its given range
    csr = gg.random_csr(300, 300, 0.03, seed, power=1.2)
    fmt = rf.build(csr, W=16, wl=[wl] * 8, S=64, split_len=split, bounds=bounds)
    check_invariants(csr, fmt)
    want_b = [0] + bounds[:-1] if bounds[-1] == 300 else [0] + bounds
    assert list(fmt["tile_col_begin"]) == want_b
    assert fmt["T"] == len(bounds)
    x = gg.uniform_f32(300, seed)
    assert np.allclose(rf.spmv_format(fmt, x), oracle.spmv(csr, x), rtol=1e-12, atol=1e-14)


def test_given_bounds_at_a_fixed_width_equal_algorithm_1_tiles():
    # bounds every W columns reproduce the fixed-width tiles exactly
    csr = gg.random_csr(400, 400, 0.02, 9, power=1.1)
    a = rf.build(csr, W=50, n_tiles=3, wl=[77] * 8, S=64, split_len=20)
    b = rf.build(csr, W=999, wl=[77] * 8, S=64, split_len=20, bounds=[50, 100, 150])
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k
    assert a["T"] == b["T"] == 3
