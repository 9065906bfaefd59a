"""How good are the runtime choices of Section 3.3 on this GPU?

For a matrix, the workload size chosen by Algorithms 2-3 (with the measured
throughput table) is compared with an exhaustive sweep of given sizes:

* the autotuned size's measured time against the best measured one (the
  paper reports the autotuned tiling within 3% of exhaustive search);
* the tile count of Algorithm 1 (1M-column tiles) against given counts;
* for every size, the model's predicted time (Eq. 1-5) against the measured
  tile-kernel time (the paper reports the model within about 20%).

Times are tile-kernel microseconds per product, from HIP events around every
launch.  Prints one JSON line per matrix.

    python -m paper_1103_2405_amd.autotune_check [--graphs rmat20,cl23] [--reps 20]
"""
from __future__ import annotations

import argparse
import json
import sys

import torch

from .tc import DeviceCsr, TiledMatrix

SWEEP = (512, 1024, 2048, 4096, 8192, 16384, 32768)
TILES = (0, 1, 2, 4, 8)


def _graph(name: str):
    import graphgen as gg
    if name == "rmat20":
        return gg.pagerank_matrix(gg.rmat(20, 16, seed=20)), "pagerank-rmat-20"
    if name == "cl23":
        return gg.pagerank_matrix(gg.chung_lu(23, 1 << 27, gamma=2.1, cap=float(1 << 20), seed=23)), \
            "pagerank-chung-lu-2^23"
    raise SystemExit("unknown graph " + name)


def measure(A: DeviceCsr, reps: int, **opts):
    tm = TiledMatrix(A, **opts)
    info = tm.info()
    wl = [int(v) for v in tm.export_format(metadata_only=True)["tile_wl"]]
    x = torch.rand(A.n_cols, device="cuda")
    y = torch.empty(A.n_rows, device="cuda")
    for _ in range(3):
        tm.spmv_internal(x, y)
    tm.set_timing(True)
    for _ in range(reps):
        tm.spmv_internal(x, y)
    t = tm.get_timing()
    tm.close()
    us = t["tile_kernel_ms"] * 1e3 / max(t["spmv_calls"], 1)
    return {"wl": wl, "n_tiles_built": info["n_tiles"], "model_us": round(info["model_us"], 1),
            "measured_us": round(us, 1), "model_over_measured": round(info["model_us"] / us, 3)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", default="rmat20,cl23")
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args(argv)
    assert torch.cuda.is_available(), "runs on the GPU"
    for name in a.graphs.split(","):
        csr, desc = _graph(name)
        A = DeviceCsr(csr)
        auto = measure(A, a.reps)
        sweep = [dict(measure(A, a.reps, wl=w), given=w) for w in SWEEP]
        best = min([auto] + sweep, key=lambda r: r["measured_us"])
        # tile count (Algorithm 1) at 1M-column tiles (4 MB of x, one XCD's L2)
        # against given counts; all with autotuned workload sizes
        W = 1 << 20
        tiles_auto = dict(measure(A, a.reps, tile_width=W), n_tiles="Algorithm 1")
        tiles = [dict(measure(A, a.reps, tile_width=W, n_tiles=t), n_tiles=t) for t in TILES]
        tbest = min([tiles_auto] + tiles, key=lambda r: r["measured_us"])
        print(json.dumps({"workload": desc, "nnz": int(A.nnz), "autotuned": auto, "sweep": sweep,
                          "best_measured_us": best["measured_us"], "best_wl": best["wl"],
                          "autotuned_over_best": round(auto["measured_us"] / best["measured_us"], 3),
                          "tile_width": W, "tiles_autotuned": tiles_auto, "tiles_sweep": tiles,
                          "tiles_autotuned_over_best": round(tiles_auto["measured_us"] / tbest["measured_us"], 3)}),
              flush=True)
        del A
        torch.cuda.empty_cache()


if __name__ == "__main__":
    sys.exit(main())
