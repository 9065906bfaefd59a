"""Offline component of the performance model (Section 3.3): measure the tile
kernel's throughput for every workload shape and write the (w, h) table that
Algorithms 2-3 read.

For one shape (w, h) the benchmark matrix has rows of exactly w entries and
the workload size is w*h, so every workload is the same w x h rectangle
(row-major when w >= h, column-major otherwise), and there are enough of them
to fill the GPU.  Columns are uniform in a window: 2^20 columns for the dense
table (a tile's x segment) and 2^23 for the sparse one (no reuse), the two
tables of Section 3.3.  Throughput is entries per microsecond of tile-kernel
time (HIP events around every launch).

The grid covers powers of two with w*h <= 32768 (the workload bound of
Section 4.4) and w or h >= 64 (one side padded to the wavefront); other grid
cells copy the nearest measured cell, so the table is complete.

    python -m paper_1103_2405_amd.tune_table [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import torch

from .tc import DEFAULT_PERF_TABLE, DeviceCsr, TiledMatrix

NG = 16
MAX_AREA = 32768


def measured_cells():
    cells = []
    for lw in range(NG):
        for lh in range(NG):
            if lw + lh > 15:
                continue
            w, h = 1 << lw, 1 << lh
            if (w >= h and w >= 64) or (h > w and h >= 64):
                cells.append((lw, lh))
    return cells


def bench_shape(lw: int, lh: int, ncols: int, target_nnz: int, reps: int, gen: torch.Generator) -> int:
    w, h = 1 << lw, 1 << lh
    area = w * h
    n_wl = max(8192, target_nnz // area)
    n_wl = min(n_wl, (64 << 20) // area + 1)
    rows = n_wl * h
    nnz = rows * w
    dev = torch.device("cuda")
    rp = torch.arange(0, rows + 1, dtype=torch.int64, device=dev) * w
    col = torch.randint(0, ncols, (nnz,), generator=gen, device=dev, dtype=torch.int32)
    val = torch.ones(nnz, dtype=torch.float32, device=dev)
    csr = DeviceCsr((rows, ncols, rp, col, val), device=dev)
    tm = TiledMatrix(csr, tile_width=ncols, n_tiles=1, wl=area, split_len=0, relabel=0, perf_table=None)
    x = torch.rand(ncols, device=dev)
    y = torch.empty(rows, device=dev)
    for _ in range(2):
        tm.spmv_internal(x, y)
    tm.set_timing(True)
    for _ in range(reps):
        tm.spmv_internal(x, y)
    t = tm.get_timing()
    tm.close()
    us = t["tile_kernel_ms"] * 1e3 / max(t["spmv_calls"], 1)
    return max(1, int(round(nnz / us)))


def fill(grid: dict) -> dict:
    out = {}
    keys = sorted(grid)
    for lw in range(NG):
        for lh in range(NG):
            if (lw, lh) in grid:
                out[(lw, lh)] = grid[(lw, lh)]
                continue
            best = min(keys, key=lambda k: (abs(k[0] - lw) + abs(k[1] - lh), k))
            out[(lw, lh)] = grid[best]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PERF_TABLE)
    ap.add_argument("--quick", action="store_true", help="fewer entries per shape")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    assert torch.cuda.is_available(), "the table is measured on the GPU"
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    target = (4 << 20) if args.quick else (32 << 20)
    tables = {}
    t0 = time.time()
    for kind, ncols in (("dense", 1 << 20), ("sparse", 1 << 23)):
        grid = {}
        for lw, lh in measured_cells():
            grid[(lw, lh)] = bench_shape(lw, lh, ncols, target, args.reps, gen)
            print("%s w=%d h=%d : %d entries/us" % (kind, 1 << lw, 1 << lh, grid[(lw, lh)]), flush=True)
        tables[kind] = fill(grid)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        f.write("# Tile-kernel throughput (entries per microsecond) per padded workload shape,\n")
        f.write("# measured by paper_1103_2405_amd/tune_table.py on %s in %.0f s.\n"
                % (torch.cuda.get_device_name(0), time.time() - t0))
        f.write("# kind log2(w) log2(h) value; unmeasured cells copy the nearest measured one\n")
        for kind in ("dense", "sparse"):
            for (lw, lh), v in sorted(tables[kind].items()):
                f.write("%s %d %d %d\n" % (kind, lw, lh, v))
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    sys.exit(main())
