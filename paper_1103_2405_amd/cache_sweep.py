"""The cache-size microbenchmark of Section 3.1 (Solution 1), on this GPU.

The paper finds the tile width by taking the column indices modulo a width
Wm, so that every x access falls in the first Wm entries, and sweeping Wm:
the SpMV time stays flat while the segment fits the cache and rises beyond
(the knee).  Here the matrix is the Chung-Lu PageRank matrix (or R-MAT 20),
each modded matrix is built as one tile (or, with --panels, in row panels
with column tiles), and the kernel time per product comes from HIP events
around every launch.

    python -m paper_1103_2405_amd.cache_sweep [--graph cl23|rmat20] [--reps 10]
        [--panels -1] [--widths 1024,8388608]

Prints one JSON line: the widths, the microseconds per product, and the
knee (the largest width within 10% of the time at the smallest width).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from .tc import DeviceCsr, TiledMatrix

WIDTHS = [1 << s for s in range(10, 24)]  # 1K .. 8M columns (4 KB .. 32 MB of x)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--graph", default="cl23")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--panels", type=int, default=0,
                    help="build with row panels (-1 automatic) instead of one tile")
    ap.add_argument("--widths", default="", help="comma-separated widths (default: 1K .. n_cols by powers of two)")
    a = ap.parse_args(argv)
    assert torch.cuda.is_available(), "runs on the GPU"
    import graphgen as gg
    if a.graph == "cl23":
        csr = gg.pagerank_matrix(gg.chung_lu(23, 1 << 27, gamma=2.1, cap=float(1 << 20), seed=23))
    else:
        csr = gg.pagerank_matrix(gg.rmat(20, 16, seed=20))
    n_rows, n_cols, rp, col, val = csr
    A = DeviceCsr(csr)
    col_d = A.col.clone()
    res = []
    widths = [int(v) for v in a.widths.split(",")] if a.widths else [w for w in WIDTHS if w <= n_cols]
    for wm in widths:
        A.col.copy_(torch.remainder(col_d, wm))
        if a.panels:
            # the benchmark's format (row panels, column tiles by Algorithm 1)
            # on the modded matrix
            tm = TiledMatrix(A, panels=a.panels)
        else:
            tm = TiledMatrix(A, tile_width=n_cols, n_tiles=1, relabel=0)
        x = torch.rand(n_cols, device="cuda")
        y = torch.empty(n_rows, device="cuda")
        for _ in range(2):
            tm.spmv_internal(x, y)
        tm.set_timing(True)
        for _ in range(a.reps):
            tm.spmv_internal(x, y)
        t = tm.get_timing()
        res.append((wm, t["tile_kernel_ms"] * 1e3 / max(t["spmv_calls"], 1)))
        if a.panels:
            inf = tm.info()
            print("   panels %d, column tiles %d" % (inf["n_panels"], inf["n_col_tiles"]), file=sys.stderr, flush=True)
        print("width %8d (%8.1f KB of x): %8.1f us" % (wm, wm * 4 / 1024, res[-1][1]), file=sys.stderr, flush=True)
        tm.close()
    base = res[0][1]
    knee = max(w for w, us in res if us <= 1.1 * base)
    print(json.dumps({"graph": a.graph, "nnz": int(A.nnz), "widths": [w for w, _ in res],
                      "us": [round(u, 1) for _, u in res], "knee_width": knee,
                      "knee_kb": knee * 4 // 1024}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
