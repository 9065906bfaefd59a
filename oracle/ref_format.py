"""Reference builder of the tiled composite format.  TEST INFRASTRUCTURE ONLY:
used by the tests to check the GPU builder element for element; the library
never imports it.

It follows the paper's preprocessing in order:
  a1 column lengths ............................ Section 3.1, Solution 2
  a2 columns sorted by decreasing length ........ Solution 2 (ties: ascending id,
     as a stable counting sort gives, Sorting Cost paragraph); square matrices
     relabel rows the same way
  a3 number of dense tiles ...................... Algorithm 1
  a4 entries bucketed by tile ................... Solution 1 (tile of W columns),
     the columns past the dense tiles forming one sparse tile (Solution 3, last
     paragraph)
  a5 rows of each tile sorted by decreasing length (ties: ascending internal row)
  a6 rows packed into workloads ................. Solution 3, Algorithm 3
  a7 padded row-major / column-major rectangles . Solution 3, Figure 1(d)

Layout of the result (all numpy arrays, see `build`):
  element (r, c) of a row-major workload sits at data_off + r * w_pad + c, of a
  column-major one at data_off + c * h_pad + r; c runs over the row's entries in
  the input CSR order; pad entries hold value +0.0 and the tile's first internal
  column; rowid holds the internal row of every workload row (-1 for pad rows).
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .autotune import RM, CM, PerfTable, choose_wl, count_tiles, partition_rows, tile_split_len


def xcd_boundaries(clen_sorted: np.ndarray, W: int, groups: int) -> list:
    """Column ranges of the XCD schedule: the head [0, W) as one tile, then the
    remaining columns cut into `groups` ranges holding equal numbers of
    entries (range g ends at the first column where the entries after W reach
    ceil(g * rest / groups))."""
    n_cols = len(clen_sorted)
    head = min(W, n_cols)
    pre = np.concatenate([[0], np.cumsum(clen_sorted[head:], dtype=np.int64)])
    rest = int(pre[-1])
    bounds = [0, head]
    for g in range(1, groups):
        need = -(-(g * rest) // groups)
        c = head + int(np.searchsorted(pre, need, side="left"))
        bounds.append(max(min(c, n_cols), bounds[-1]))
    bounds.append(n_cols)
    return bounds


def panel_weights(n_rows: int, irow: np.ndarray, ctile: np.ndarray, csplit: Sequence[int]) -> np.ndarray:
    """Entries of each internal row that stay with the row: the row's segment
    in a column tile counts unless the tile's split length cuts it into chunks
    (chunks are not tied to a panel)."""
    if irow.size == 0:
        return np.zeros(n_rows, np.int64)
    key = ctile.astype(np.int64) * n_rows + irow
    u, cnt = np.unique(key, return_counts=True)
    t, r = u // n_rows, u % n_rows
    sp = np.asarray(csplit, np.int64)[t]
    keep = (sp == 0) | (cnt <= sp)
    return np.bincount(r[keep], weights=cnt[keep], minlength=n_rows).astype(np.int64)


def panel_bounds(weight: np.ndarray, panels: int, max_rows: int) -> list:
    """Row panels: contiguous ranges of internal rows, panel p ending at the
    first row where the running weight reaches ceil((p+1) total / panels),
    each at least one row and at most max_rows; rows left after `panels`
    panels go into further panels of max_rows."""
    n = len(weight)
    if max_rows <= 0:
        raise ValueError("panel_rows must be positive")
    pre = np.concatenate([[0], np.cumsum(weight, dtype=np.int64)])
    total = int(pre[-1])
    b = [0]
    for p in range(panels):
        if b[-1] >= n:
            break
        tgt = -(-((p + 1) * total) // panels)
        lb = int(np.searchsorted(pre, tgt, side="left"))
        b.append(min(max(lb, b[-1] + 1), b[-1] + max_rows, n))
    while b[-1] < n:
        b.append(min(b[-1] + max_rows, n))
    return b


def build(csr, W: int, n_tiles: int = -1, wl: Optional[Sequence[int]] = None, S: int = 64,
          split_len: int = -1, camping_pad: bool = False, relabel: Optional[bool] = None,
          table: Optional[PerfTable] = None, max_act_warp: int = 8192, xcd_groups: int = 0,
          coo: bool = False, bounds: Optional[Sequence[int]] = None, panels: int = 0,
          panel_rows: int = 0, panel_waves: int = 16) -> dict:
    n_rows, n_cols, rp, col, val = csr
    rp = np.asarray(rp, np.int64)
    col = np.asarray(col, np.int32)
    val = np.asarray(val, np.float32)
    nnz = int(rp[-1]) if n_rows > 0 else 0
    if W <= 0:
        raise ValueError("W must be positive")

    # a1: column lengths
    clen = np.bincount(col, minlength=n_cols).astype(np.int64)
    # a2: stable sort by decreasing length
    cperm = np.argsort(-clen, kind="stable").astype(np.int64)
    cpos = np.empty(n_cols, np.int64)
    cpos[cperm] = np.arange(n_cols)
    if relabel is None:
        relabel = n_rows == n_cols
    rmap = cpos.copy() if relabel else np.arange(n_rows, dtype=np.int64)

    # a3: Algorithm 1
    if bounds:
        # given boundaries: dense tiles [0, b0), [b0, b1), ..., then the
        # columns past the last bound as the sparse tile
        b = [0] + [int(v) for v in bounds]
        if any(b[i + 1] <= b[i] for i in range(len(b) - 1)) or b[-1] > n_cols:
            raise ValueError("bounds must increase within (0, n_cols]")
        ranges = [(b[i], b[i + 1]) for i in range(len(b) - 1)]
        if b[-1] < n_cols:
            ranges.append((b[-1], n_cols))
        T = len(bounds)
    elif xcd_groups > 0:
        # MI355X schedule: hot head tile, then column ranges of equal entries
        b = xcd_boundaries(clen[cperm], W, xcd_groups)
        ranges = [(b[i], b[i + 1]) for i in range(len(b) - 1)]
        T = 1
    else:
        NT = -(-n_cols // W)
        T = min(n_tiles, NT) if n_tiles >= 0 else count_tiles(clen[cperm], W)
        ranges = [(t * W, min((t + 1) * W, n_cols)) for t in range(T)]
        if T * W < n_cols:
            ranges.append((T * W, n_cols))
    ntiles = len(ranges)
    starts = np.asarray([r[0] for r in ranges[1:]], np.int64)

    # a4: stable bucketing of entries by tile
    row_of = np.repeat(np.arange(n_rows, dtype=np.int64), np.diff(rp))
    icol = cpos[col] if nnz else np.zeros(0, np.int64)
    tile_of = np.searchsorted(starts, icol, side="right") if nnz else np.zeros(0, np.int64)
    NT = ntiles  # column tiles
    ccount = np.bincount(tile_of, minlength=NT) if nnz else np.zeros(NT, np.int64)
    csplit = [tile_split_len(split_len, int(ccount[t]), max_act_warp, S) for t in range(NT)]
    pb = None
    if panels > 0:
        # row panels: tile g = panel * NT + column tile
        pb = panel_bounds(panel_weights(n_rows, rmap[row_of], tile_of, csplit), panels, panel_rows)
        prow = np.searchsorted(pb, rmap[row_of], side="right") - 1 if nnz else np.zeros(0, np.int64)
        tile_of = prow * NT + tile_of
        ranges = [ranges[g % NT] for g in range((len(pb) - 1) * NT)]
        ntiles = len(ranges)
    order = np.argsort(tile_of, kind="stable")
    tcount = np.bincount(tile_of, minlength=ntiles) if nnz else np.zeros(ntiles, np.int64)
    tstart = np.concatenate([[0], np.cumsum(tcount)])

    tile_row_off = [0]
    rows_sorted, rows_len = [], []
    wl_used, split_used = [], []
    W_ = {k: [] for k in ("tile", "layout", "w", "w_pad", "h_pad", "row_begin", "n_rows",
                          "chunk", "n_chunks")}
    seg_lists = []  # per tile: (sorted segment starts into `order`, lengths)
    for t in range(ntiles):
        pos = order[tstart[t]:tstart[t + 1]]
        rows = row_of[pos]
        if len(rows):
            head = np.concatenate([[True], rows[1:] != rows[:-1]])
            sstart = np.flatnonzero(head)
            slen = np.diff(np.concatenate([sstart, [len(rows)]]))
            srow = rows[sstart]
        else:
            sstart = slen = srow = np.zeros(0, np.int64)
        # a5: sort rows by (decreasing length, increasing internal row id)
        o = np.lexsort((rmap[srow], -slen))
        sstart, slen, srow = sstart[o], slen[o], srow[o]
        rows_sorted.append(rmap[srow])
        rows_len.append(slen)
        tile_row_off.append(tile_row_off[-1] + len(srow))
        seg_lists.append((tstart[t] + sstart, slen, srow))
    for t in range(ntiles):
        slen = seg_lists[t][1]
        # a6: workload size and partition
        kind = "dense" if t % NT < T else "sparse"
        split_t = csplit[t % NT]
        split_used.append(split_t)
        if wl is not None:
            WLt = int(wl[t])
        elif table is not None:
            # with row panels a panel's tile is tuned for the wavefronts of its workgroup
            WLt = choose_wl(slen.tolist(), int(tcount[t]), table, kind, panel_waves if pb is not None else max_act_warp,
                            S, split_t)
        else:
            raise ValueError("give wl or a table")
        wl_used.append(WLt)
        for p in partition_rows(slen.tolist(), WLt, S, split_t):
            layout, w, w_pad, h_pad, rb, nr, ch, nch = p
            for k, v in zip(("tile", "layout", "w", "w_pad", "h_pad", "row_begin", "n_rows",
                             "chunk", "n_chunks"),
                            (t, layout, w, w_pad, h_pad, rb + tile_row_off[t], nr, ch, nch)):
                W_[k].append(v)

    wlarr = {k: np.asarray(v, np.int64) for k, v in W_.items()}
    nwl = len(wlarr["tile"])
    area = wlarr["w_pad"] * wlarr["h_pad"]
    extra = np.where(camping_pad & (area % 512 == 0), 64, 0) if nwl else np.zeros(0, np.int64)
    size = area + extra
    data_off = np.concatenate([[0], np.cumsum(size)])[:nwl] if nwl else np.zeros(0, np.int64)
    nnz_pad = int(size.sum()) if nwl else 0
    rid_cnt = wlarr["h_pad"]  # row-major: h rows; column-major: padded rows; chunk: 1
    rowid_off = np.concatenate([[0], np.cumsum(rid_cnt)])[:nwl] if nwl else np.zeros(0, np.int64)
    n_rowid = int(rid_cnt.sum()) if nwl else 0

    # a7: pack
    tile_first = np.asarray([r[0] for r in ranges], np.int64)
    idx_out = np.repeat(tile_first[wlarr["tile"]], size).astype(np.int32) if nwl else np.zeros(0, np.int32)
    val_out = np.zeros(nnz_pad, np.float32)
    rowid = np.full(n_rowid, -1, np.int32)
    rows_sorted_all = np.concatenate(rows_sorted) if ntiles else np.zeros(0, np.int64)
    seg_start_all = np.concatenate([s[0] for s in seg_lists]) if ntiles else np.zeros(0, np.int64)
    seg_len_all = np.concatenate([s[1] for s in seg_lists]) if ntiles else np.zeros(0, np.int64)

    for j in range(nwl):
        rb, nr = int(wlarr["row_begin"][j]), int(wlarr["n_rows"][j])
        off, wp, hp = int(data_off[j]), int(wlarr["w_pad"][j]), int(wlarr["h_pad"][j])
        lay, ch = int(wlarr["layout"][j]), int(wlarr["chunk"][j])
        ro = int(rowid_off[j])
        if ch >= 0:
            s0 = int(seg_start_all[rb])
            c0 = ch * split_used[int(wlarr["tile"][j])]
            cw = int(wlarr["w"][j])
            src = order[s0 + c0: s0 + c0 + cw]
            idx_out[off:off + cw] = cpos[col[src]]
            val_out[off:off + cw] = val[src]
            rowid[ro] = rows_sorted_all[rb]
            continue
        rowid[ro:ro + nr] = rows_sorted_all[rb:rb + nr]
        lens = seg_len_all[rb:rb + nr]
        starts = seg_start_all[rb:rb + nr]
        tot = int(lens.sum())
        if tot == 0:
            continue
        r_of = np.repeat(np.arange(nr), lens)
        c_of = np.arange(tot) - np.repeat(np.cumsum(lens) - lens, lens)
        src = order[np.repeat(starts, lens) + c_of]
        dest = off + (r_of * wp + c_of if lay == RM else c_of * hp + r_of)
        idx_out[dest] = cpos[col[src]]
        val_out[dest] = val[src]

    extra = {}
    if coo:
        # TILE-COO (Section 3.1, Observation 3): each tile's entries in
        # coordinate form, in the bucketed order (tiles ascending, rows ascending
        # inside a tile, input order inside a row).  A row whose first tile is
        # an earlier one carries bit 30 (the kernel adds to y instead of storing).
        rows_b = row_of[order]
        tile_b = tile_of[order]
        first_tile = np.full(n_rows, np.iinfo(np.int64).max, np.int64)
        np.minimum.at(first_tile, rows_b, tile_b)
        flag = np.where(first_tile[rows_b] < tile_b, 1 << 30, 0)
        extra = dict(coo_row=(rmap[rows_b] | flag).astype(np.int32), coo_col=icol[order].astype(np.int32),
                     coo_val=val[order].astype(np.float32))
    return dict(
        **extra,
        n_rows=n_rows, n_cols=n_cols, nnz=nnz, W=W, S=S, split_len=split_len, T=T, xcd_groups=xcd_groups, bounds=list(bounds) if bounds else None,
        tile_split=np.asarray(split_used, np.int64),
        n_tiles_total=ntiles, relabel=bool(relabel), n_col_tiles=NT,
        panel_begin=None if pb is None else np.asarray(pb, np.int64), panel_rows=panel_rows, panel_waves=panel_waves,
        clen=clen, cperm=cperm.astype(np.int32), cpos=cpos.astype(np.int32),
        rowmap=rmap.astype(np.int32),
        tile_col_begin=np.asarray([r[0] for r in ranges], np.int64),
        tile_col_end=np.asarray([r[1] for r in ranges], np.int64),
        tile_nnz=tcount.astype(np.int64), tile_wl=np.asarray(wl_used, np.int64),
        tile_row_off=np.asarray(tile_row_off, np.int64),
        rows_sorted=rows_sorted_all.astype(np.int32), rows_len=seg_len_all.astype(np.int64),
        wl_tile=wlarr["tile"], wl_layout=wlarr["layout"], wl_w=wlarr["w"],
        wl_w_pad=wlarr["w_pad"], wl_h_pad=wlarr["h_pad"], wl_row_begin=wlarr["row_begin"],
        wl_n_rows=wlarr["n_rows"], wl_chunk=wlarr["chunk"], wl_n_chunks=wlarr["n_chunks"],
        wl_data_off=data_off.astype(np.int64), wl_rowid_off=rowid_off.astype(np.int64),
        nnz_pad=nnz_pad, idx=idx_out, val=val_out, rowid=rowid,
    )


def decode_coo(fmt: dict):
    """Round trip: the (original row, original column, value) entries the
    format stores, sorted, for comparison with the input CSR."""
    cperm = fmt["cperm"].astype(np.int64)
    rowmap = fmt["rowmap"].astype(np.int64)
    inv_row = np.empty(len(rowmap), np.int64)
    inv_row[rowmap] = np.arange(len(rowmap))
    R, C, V = [], [], []
    for j in range(len(fmt["wl_tile"])):
        rb, nr = int(fmt["wl_row_begin"][j]), int(fmt["wl_n_rows"][j])
        off, wp, hp = int(fmt["wl_data_off"][j]), int(fmt["wl_w_pad"][j]), int(fmt["wl_h_pad"][j])
        lay, ch = int(fmt["wl_layout"][j]), int(fmt["wl_chunk"][j])
        if ch >= 0:
            cw = int(fmt["wl_w"][j])
            R.append(np.full(cw, fmt["rows_sorted"][rb], np.int64))
            C.append(fmt["idx"][off:off + cw].astype(np.int64))
            V.append(fmt["val"][off:off + cw])
            continue
        for r in range(nr):
            L = int(fmt["rows_len"][rb + r])
            cs = np.arange(L)
            pos = off + (r * wp + cs if lay == RM else cs * hp + r)
            R.append(np.full(L, fmt["rows_sorted"][rb + r], np.int64))
            C.append(fmt["idx"][pos].astype(np.int64))
            V.append(fmt["val"][pos])
    if not R:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.float32)
    r = inv_row[np.concatenate(R)]
    c = cperm[np.concatenate(C)]
    v = np.concatenate(V)
    o = np.lexsort((v.view(np.uint32), c, r))
    return r[o], c[o], v[o]


def spmv_format(fmt: dict, x: np.ndarray) -> np.ndarray:
    """y = A x evaluated from the format (decode, then FP64 sums): checks the
    format's semantics on the CPU without any GPU."""
    r, c, v = decode_coo(fmt)
    y = np.zeros(fmt["n_rows"], np.float64)
    np.add.at(y, r, v.astype(np.float64) * x.astype(np.float64)[c])
    return y
