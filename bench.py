"""Benchmark of the tiled composite SpMV hot path on one MI355X.

Workload (default): a Chung-Lu power-law graph with 2^23 nodes and 2^27
distinct edges (in/out-degree exponent 2.1, degrees capped at 2^20, node ids
randomly permuted), PageRank matrix M = W^T with values fl32(1/outdeg).

One step = the whole hot path on that input, which is resident in HBM before
the timed region starts:
    build_tiled(M)      column lengths, column sort, tile count, bucketing,
                        per-tile row sort, workload sizes, pack
    pagerank(100 it.)   100 tiled SpMVs with the fused PageRank update
    destroy
value = 100 x (8 nnz + 4 (n_rows + n_cols)) bytes per step / step time, in
GB/s (whole step, build included).  The roofline object reports the tile
SpMV kernel alone, from HIP events around every launch in the timed region.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpMV GB/s & % HBM peak; batched RWR queries/s vs plain SpMV loop"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    import graphgen as gg
    t0 = time.time()
    if name == "cl23":
        g = gg.chung_lu(23, 1 << 27, gamma=2.1, cap=float(1 << 20), seed=23)
        desc = {"workload": "pagerank-chung-lu-2^23", "nodes": g.n, "edges": g.m, "gamma": 2.1,
                "degree_cap": 1 << 20, "ids_permuted": True, "pagerank_iters": 100, "seed": 23}
    elif name == "rmat20":
        g = gg.rmat(20, 16, seed=20)
        desc = {"workload": "pagerank-rmat-20", "nodes": g.n, "edges": g.m, "edge_factor": 16,
                "abcd": [0.57, 0.19, 0.19, 0.05], "pagerank_iters": 100, "seed": 20}
    elif name == "rmat14":
        g = gg.rmat(14, 16, seed=14)
        desc = {"workload": "pagerank-rmat-14", "nodes": g.n, "edges": g.m, "edge_factor": 16,
                "abcd": [0.57, 0.19, 0.19, 0.05], "pagerank_iters": 100, "seed": 14}
    else:
        raise SystemExit("unknown workload " + name)
    csr = gg.pagerank_matrix(g)
    log("workload %s: n=%d nnz=%d generated in %.1fs" % (name, g.n, csr[3].size, time.time() - t0))
    return csr, desc


def cpu_baseline(csr, budget_s: float):
    """The oracle's FP64 PageRank on the host cores, on a bounded number of iterations."""
    import oracle
    n, _, rp, col, val = csr
    nbytes = 8 * col.size + 4 * (n + n)
    t0 = time.time()
    oracle.pagerank(csr, 0.85, 0.0, 3)
    one = (time.time() - t0) / 3  # includes the call's setup: errs on the short side
    iters = max(1, min(100, int(budget_s / max(one, 1e-3))))
    t0 = time.time()
    oracle.pagerank(csr, 0.85, 0.0, iters)
    dt = time.time() - t0
    cores = oracle.num_threads()
    # one core, on a short sample of the same iteration
    oracle.set_threads(1)
    t0 = time.time()
    oracle.pagerank(csr, 0.85, 0.0, 2)
    one_core = 2 * nbytes / (time.time() - t0) / 1e9
    oracle.set_threads(cores)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(iters * nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d FP64 PageRank iterations of the same matrix (one CSR SpMV + update each), "
                      "%.1f s; same byte formula" % (iters, dt),
            "one_core_value": round(one_core, 3), "one_core_sample": "2 iterations (setup included)",
            "cpu_model": model}


def rwr_batched(c: float = 0.85, tol: float = 1e-6, ks=(1, 8, 32, 64, 128)):
    """Batched RWR (multi-RHS SpMM) on the symmetrised R-MAT scale-20 graph:
    queries/s for k one-hot restart vectors solved together to an L1 change of
    tol, against k = 32 sequential single-query solves with (a) PyTorch's
    sparse CSR matrix-vector product and (b) the tiled single-vector SpMV."""
    import torch
    import graphgen as gg
    from paper_1103_2405_amd import DeviceCsr, TiledMatrix
    g = gg.rmat(20, 16, seed=20)
    W = gg.rwr_matrix(g)
    seeds = gg.rwr_seeds(g, max(ks), 40)
    A = DeviceCsr(W)
    tm = TiledMatrix(A)
    out = {"graph": "symmetrised rmat-20", "nnz": int(A.nnz), "c": c, "tol": tol}
    for k in ks:
        tm.rwr(seeds[:k], c, tol, 500, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, it, res = tm.rwr(seeds[:k], c, tol, 500, 10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["k%d" % k] = {"queries_per_s": round(k / dt, 2), "iters": it, "ms": round(dt * 1e3, 2)}
    # (b) k sequential tiled single-vector solves (k = 32)
    k = 32
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(k):
        tm.rwr(seeds[q:q + 1], c, tol, 500, 10)
    torch.cuda.synchronize()
    tiled_seq = k / (time.perf_counter() - t0)
    n = A.n_rows

    def plain_loop(spmv):
        """k = 32 sequential single-query solves: y = A r by `spmv`, the RWR
        update and the residual (checked every 10 iterations) by torch."""
        r = torch.empty(n, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(k):
            s = int(seeds[q])
            r.zero_()
            r[s] = 1.0
            for it in range(500):
                y = spmv(r)
                y.mul_(c)
                y[s] += 1.0 - c
                d = float((y - r).abs().sum()) if (it + 1) % 10 == 0 else 1.0
                r = y
                if d <= tol:
                    break
        torch.cuda.synchronize()
        return k / (time.perf_counter() - t0)

    # (a) PyTorch's sparse CSR matrix-vector product (the ROCm sparse library)
    try:
        Wt = torch.sparse_csr_tensor(torch.from_numpy(W[2].astype(np.int32)).cuda(),
                                     torch.from_numpy(W[3]).cuda(), torch.from_numpy(W[4]).cuda(), size=(n, n))
        torch_seq = plain_loop(lambda r: torch.mv(Wt, r))
        del Wt
    except Exception as e:  # report, do not fail the benchmark
        log("torch sparse CSR baseline unavailable:", repr(e))
        torch_seq = None
    b = out["k32"]["queries_per_s"]
    out.update(tiled_loop_queries_per_s=round(tiled_seq, 2),
               torch_csr_loop_queries_per_s=None if torch_seq is None else round(torch_seq, 2),
               torch_csr_note="PyTorch sparse CSR (the ROCm sparse library): context only, not a target",
               speedup_k32_vs_tiled_loop=round(b / tiled_seq, 2),
               speedup_k32_vs_torch_csr_loop=None if torch_seq is None else round(b / torch_seq, 2))
    tm.close()
    return out


def rwr_multi_graph(c: float = 0.85, iters: int = 30, n_graphs: int = 32):
    """RWR with one query on each of 32 independent R-MAT graphs (graph g:
    seed 4000 + g, scale uniform in 10..16, edge factor uniform in 8..32),
    30 iterations each: all graphs per launch (captured once in a HIP graph,
    and eagerly) against the graphs one after another with the single-graph
    driver."""
    import torch
    import graphgen as gg
    from paper_1103_2405_amd import DeviceCsr, TiledMatrix, rwr_multi
    scales = 10 + gg.uniform_int(n_graphs, 7, 4000)
    efs = 8 + gg.uniform_int(n_graphs, 25, 4001)
    mats, seeds, nodes, nnz = [], [], 0, 0
    for g in range(n_graphs):
        G = gg.rmat(int(scales[g]), int(efs[g]), seed=4000 + g)
        W = gg.rwr_matrix(G)
        mats.append(TiledMatrix(DeviceCsr(W)))
        seeds.append(int(gg.rwr_seeds(G, 1, 4100 + g)[0]))
        nodes += G.n
        nnz += int(W[3].size)
    out = {"graphs": n_graphs, "nodes": nodes, "nnz": nnz, "iters": iters, "c": c}

    def timed(f, reps=3):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    out["multi_graph_ms"] = round(timed(lambda: rwr_multi(mats, seeds, c, 0.0, iters, iters, graph=True)), 3)
    out["multi_eager_ms"] = round(timed(lambda: rwr_multi(mats, seeds, c, 0.0, iters, iters, graph=False)), 3)

    def seq():
        for m, s in zip(mats, seeds):
            m.rwr([s], c, 0.0, iters, iters)

    out["sequential_ms"] = round(timed(seq), 3)
    out["speedup_vs_sequential"] = round(out["sequential_ms"] / min(out["multi_graph_ms"], out["multi_eager_ms"]), 2)
    for m in mats:
        m.close()
    return out


def diff_rwr(K: int = 30, every: int = 6, reps: int = 3):
    """Differentiable RWR on the symmetrised R-MAT scale-20 graph: edge weights
    softplus(theta . f_e) with 4 features per entry, column-normalised; loss
    = -sum of log scores of 16 target nodes after K iterations from one seed.
    Times the forward (weights, both builds, K iterations with checkpoints)
    and the backward (adjoint pass and the chain to theta)."""
    import torch
    import graphgen as gg
    from paper_1103_2405_amd.rwr_grad import EdgeWeightedRWR
    g = gg.rmat(20, 16, seed=20)
    n, _, rp, col, _ = gg.rwr_matrix(g)
    feats = gg.normal_f32(len(col) * 4, 21).reshape(len(col), 4)
    seed = int(gg.rwr_seeds(g, 1, 22)[0])
    targets = torch.as_tensor(gg.rwr_seeds(g, 16, 23).astype(np.int64)).cuda()
    model = EdgeWeightedRWR((n, n, rp, col), feats, seed, 0.85, K, every=every)
    theta = torch.tensor([0.4, -0.3, 0.2, 0.1], dtype=torch.float64, requires_grad=True)
    fw, bw = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        scores = model.scores(theta)
        loss = -torch.log(scores[targets].double()).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        theta.grad = None
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
    model.close()
    return {"graph": "symmetrised rmat-20", "nnz": int(len(col)), "features": 4, "iters": K,
            "checkpoint_every": every, "targets": 16, "loss": round(loss.item(), 6),
            "grad": [round(float(v), 6) for v in theta.grad], "forward_ms": round(min(fw) * 1e3, 2),
            "backward_ms": round(min(bw) * 1e3, 2)}


def rmat20_drivers(tol: float = 1e-6):
    """R-MAT scale 20 (1,048,576 nodes, edge factor 16): one SpMV and PageRank,
    HITS and one-query RWR run to an L1 change of tol (checked every 5
    iterations), each on its own tiled build; SpMV and PageRank also with
    automatic row panels."""
    import torch
    import graphgen as gg
    from paper_1103_2405_amd import DeviceCsr, TiledMatrix
    g = gg.rmat(20, 16, seed=20)
    out = {"graph": "rmat-20", "tol": tol}

    def timed(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    A = DeviceCsr(gg.pagerank_matrix(g))
    tm = TiledMatrix(A)
    x = torch.rand(A.n_cols, device="cuda")
    y = torch.empty(A.n_rows, device="cuda")
    _, ms = timed(lambda: [tm.spmv_internal(x, y) for _ in range(20)])
    nbytes = 8 * A.nnz + 4 * (A.n_rows + A.n_cols)
    out["spmv"] = {"nnz": int(A.nnz), "us": round(ms * 1e3 / 20, 1), "gbps": round(nbytes / (ms / 20 * 1e6), 1),
                   "n_tiles": tm.info()["n_tiles"], "wl": [int(v) for v in tm.export_format(True)["tile_wl"]]}
    (p, it, res), ms = timed(lambda: tm.pagerank(0.85, tol, 1000, 5))
    out["pagerank"] = {"iters": it, "resid": res, "ms": round(ms, 2)}
    tm.close()
    # the same with automatic row panels (the benchmark's format)
    tp = TiledMatrix(A, panels=-1)
    _, ms = timed(lambda: [tp.spmv_internal(x, y) for _ in range(20)])
    inf = tp.info()
    out["spmv_panels"] = {"us": round(ms * 1e3 / 20, 1), "gbps": round(nbytes / (ms / 20 * 1e6), 1),
                          "n_panels": inf["n_panels"], "n_col_tiles": inf["n_col_tiles"]}
    (p, it, res), ms = timed(lambda: tp.pagerank(0.85, tol, 1000, 5))
    out["pagerank_panels"] = {"iters": it, "resid": res, "ms": round(ms, 2)}
    tp.close()
    H = TiledMatrix(DeviceCsr(gg.hits_matrix(g)))
    (a, h, it, res), ms = timed(lambda: H.hits(tol, 1000, 5))
    out["hits"] = {"nnz": int(H.nnz), "iters": it, "resid": res, "ms": round(ms, 2)}
    H.close()
    R = TiledMatrix(DeviceCsr(gg.rwr_matrix(g)))
    s = gg.rwr_seeds(g, 1, 40)
    (r, it, res), ms = timed(lambda: R.rwr(s, 0.85, tol, 1000, 5))
    out["rwr"] = {"nnz": int(R.nnz), "iters": it, "resid": res, "ms": round(ms, 2)}
    R.close()
    return out


def kernel_compare(A_cl23=None, reps: int = 20):
    """TILE-COMPOSITE against TILE-COO (the paper's two kernels, Section 4):
    microseconds per product and effective GB/s (the metric's byte count) on
    power-law and non-power-law matrices, including the dense 2000 x 2000
    case of Section 4."""
    import torch
    import graphgen as gg
    from paper_1103_2405_amd import DeviceCsr, TiledMatrix
    mats = []
    if A_cl23 is not None:
        mats.append(("pagerank-chung-lu-2^23", A_cl23))
    mats.append(("pagerank-rmat-20", DeviceCsr(gg.pagerank_matrix(gg.rmat(20, 16, seed=20)))))
    n = 1 << 20  # uniform random rows of 16 entries (not power-law)
    rp = np.arange(n + 1, dtype=np.int64) * 16
    mats.append(("uniform-random-2^20x16", DeviceCsr((n, n, rp, gg.uniform_int(n * 16, n, 77).astype(np.int32),
                                                      gg.uniform_f32(n * 16, 78)))))
    d = 2000
    mats.append(("dense-2000", DeviceCsr((d, d, np.arange(d + 1, dtype=np.int64) * d,
                                          np.tile(np.arange(d, dtype=np.int32), d), gg.uniform_f32(d * d, 2000)))))
    out = {}
    for name, A in mats:
        nbytes = 8 * A.nnz + 4 * (A.n_rows + A.n_cols)
        row = {"nnz": int(A.nnz)}
        for kernel in ("composite", "coo"):
            tm = TiledMatrix(A, kernel=kernel)
            x = torch.rand(A.n_cols, device="cuda")
            y = torch.empty(A.n_rows, device="cuda")
            for _ in range(3):
                tm.spmv_internal(x, y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                tm.spmv_internal(x, y)
            torch.cuda.synchronize()
            us = (time.perf_counter() - t0) / reps * 1e6
            row[kernel] = {"us": round(us, 1), "gbps": round(nbytes / us / 1e3, 1)}
            tm.close()
        out[name] = row
    return out


def attainable_bandwidth(dev, gib: int = 2, reps: int = 10):
    """The streaming-read rate the product kernels can reach on this GPU, next
    to the nominal HBM peak: the library's own read kernel (tc_stream_read:
    16-byte non-temporal loads, four in flight per thread) over `gib` GiB,
    timed with events on the launch stream; median of reps."""
    import torch
    from paper_1103_2405_amd.tc import STREAM_SINK_FLOATS, stream_read
    n = (gib << 30) // 4
    a = torch.rand(n, device=dev)
    sink = torch.empty(STREAM_SINK_FLOATS, device=dev)
    stream_read(a, sink)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        stream_read(a, sink)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    res = {"read_gbps": round(4 * n / (float(np.median(ts)) / 1e3) / 1e9, 1), "bytes": 4 * n,
           "kernel": "k_stream_read (tc_stream_read)"}
    del a, sink
    torch.cuda.empty_cache()
    return res


def attainable_gather(dev, window: int = 1 << 19, n: int = 1 << 27, reps: int = 10):
    """The random-gather rate the product kernels can reach: the library's
    gather kernel (tc_gather_read: coalesced index and value streams, one
    gather of x per entry, eight in flight per lane) over n entries whose
    indices are uniform in a window of `window` floats (the panel pass's
    column tile: 2 MB, held by each XCD's L2); median of reps, in gathers/s."""
    import torch
    from paper_1103_2405_amd.tc import STREAM_SINK_FLOATS, gather_read
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    idx = torch.randint(0, window, (n,), device=dev, dtype=torch.int32, generator=gen)
    val = torch.rand(n, device=dev, generator=gen)
    x = torch.rand(window, device=dev, generator=gen)
    sink = torch.empty(STREAM_SINK_FLOATS, device=dev)
    gather_read(x, idx, val, sink)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gather_read(x, idx, val, sink)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del idx, val, x, sink
    torch.cuda.empty_cache()
    return {"gather_gps": round(n / (float(np.median(ts)) / 1e3) / 1e9, 1), "gather_window_floats": window,
            "gather_entries": n, "gather_kernel": "k_gather_read (tc_gather_read)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--workload", default="cl23")
    ap.add_argument("--tile-width", type=int, default=0)
    ap.add_argument("--split-len", type=int, default=-1)
    ap.add_argument("--panels", type=int, default=-1,
                    help="row panels: -1 automatic (default), 0 none (one launch per tile), P > 0 that many")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-timing", action="store_true", help="skip the per-launch kernel timing")
    ap.add_argument("--no-rwr", action="store_true", help="skip the batched RWR measurement")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (scale reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1103_2405_amd import DeviceCsr, TiledMatrix, csr_spmv, load_library

    load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    csr, desc = make_workload(args.workload)
    n = csr[0]
    nnz = csr[3].size
    spmv_bytes = 8 * nnz + 4 * (csr[0] + csr[1])
    A = DeviceCsr(csr, device=dev)
    p_out = torch.empty(n, dtype=torch.float32, device=dev)
    perf_table = "default"

    def step(timing: bool):
        tm = TiledMatrix(A, tile_width=args.tile_width, split_len=args.split_len, perf_table=perf_table,
                         panels=args.panels)
        if timing:
            tm.set_timing(True)
        tm.pagerank(0.85, 0.0, args.iters, out=p_out)
        tinfo = tm.get_timing() if timing else None
        info = tm.info()
        tm.close()
        return info, tinfo

    # warmup
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()

    # timed steps
    timing = not args.no_timing
    t0 = time.perf_counter()
    infos, marks = [], []
    for _ in range(args.steps):
        infos.append(step(timing))
        marks.append(time.perf_counter())  # each step ends synchronised (PageRank reads its residual)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_step = np.diff(np.asarray([t0] + marks)) * 1e3
    ms_per_step = dt / args.steps * 1e3
    value = args.iters * spmv_bytes / (ms_per_step / 1e3) / 1e9
    info = infos[-1][0]

    roofline = None
    if timing:
        tot_ms = sum(t["tile_kernel_ms"] for _, t in infos)
        launches = sum(t["tile_launches"] for _, t in infos)
        calls = sum(t["spmv_calls"] for _, t in infos)
        per_launch_bytes = spmv_bytes * calls / max(launches, 1)
        avg_ms = tot_ms / max(launches, 1)
        achieved = per_launch_bytes / (avg_ms / 1e3) / 1e9
        from paper_1103_2405_amd.profsum import read_traffic
        kname = "k_panel_spmv" if info["n_panels"] > 0 else "k_tile_spmv"
        traffic = read_traffic(os.path.join(ROOT, "profiles", "%s_%s_pagerank_counters.txt" % (kname, args.workload)))
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    # the row-panel pass (one launch per product), or the tile kernel with the fused update
                    "kernel": kname if info["n_panels"] > 0 else "k_tile_spmv_pr",
                    "avg_launch_us": round(avg_ms * 1e3, 2),
                    "launches_per_spmv": round(launches / max(calls, 1), 2),
                    "bytes_per_launch": int(per_launch_bytes)}

    # separate measurements (not part of value): PageRank alone and the plain CSR baseline
    tm = TiledMatrix(A, tile_width=args.tile_width, split_len=args.split_len, perf_table=perf_table,
                     panels=args.panels)
    tm.pagerank(0.85, 0.0, 5, out=p_out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm.pagerank(0.85, 0.0, args.iters, out=p_out)
    torch.cuda.synchronize()
    pr_ms = (time.perf_counter() - t1) * 1e3
    x = torch.rand(n, device=dev)
    y = torch.empty(n, device=dev)
    csr_spmv(A, x, y)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):  # CSR-vector: one wavefront per row, the longest (562K entries) alone
        csr_spmv(A, x, y)
    torch.cuda.synchronize()
    csr_ms = (time.perf_counter() - t1) * 1e3 / 3
    # entries of the panel pass whose gathers read the LDS-staged head tile
    # (column tile 0 of every panel) and those that gather from global memory
    split = None
    if info["n_panels"] > 0:
        fm = tm.export_format(metadata_only=True)
        tn = np.asarray(fm["tile_nnz"], np.int64)
        nct = info["n_col_tiles"]
        head = int(tn[::nct].sum())
        split = {"lds_entries": head, "global_gathers": int(tn.sum()) - head}
    tm.close()

    if args.probe_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    attainable = None if args.no_rwr else attainable_bandwidth(dev)
    if attainable is not None:
        attainable.update(attainable_gather(dev))
        if split is not None:
            # a lower bound of the panel pass from the two measured rates: its
            # global gathers at the gather rate (their index and value streams
            # included), the head tile's entries streamed at the read rate
            attainable["panel_pass"] = dict(split, floor_us=round(
                split["global_gathers"] / (attainable["gather_gps"] * 1e3) +
                8 * split["lds_entries"] / (attainable["read_gbps"] * 1e3), 1))

    kernels = None if args.no_rwr else kernel_compare(A)
    if kernels:
        log("kernels:", json.dumps(kernels))
    drivers = None if args.no_rwr else rmat20_drivers()
    if drivers:
        log("rmat-20 drivers:", json.dumps(drivers))

    rwr = None
    if not args.no_rwr:
        del A
        torch.cuda.empty_cache()
        rwr = rwr_batched()
        rwr["multi_graph"] = rwr_multi_graph()
        rwr["differentiable"] = diff_rwr()
        log("batched rwr:", json.dumps(rwr))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(csr, args.cpu_budget)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(desc, step="build_tiled + %d PageRank iterations + destroy" % args.iters,
                       tile_width=info["tile_width"], n_tiles=info["n_tiles"], n_panels=info["n_panels"],
                       n_col_tiles=info["n_col_tiles"], panel_rows=info["panel_rows"],
                       n_workloads=info["n_workloads"], nnz_pad=info["nnz_pad"]),
        "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "step_ms": {"min": round(float(per_step.min()), 3), "median": round(float(np.median(per_step)), 3),
                    "max": round(float(per_step.max()), 3)},
        "accumulate": "f64",
        "build_ms": round(info["build_us"] / 1e3, 3),
        "pagerank_ms": round(pr_ms, 3),
        "pagerank_spmv_gbps": round(args.iters * spmv_bytes / (pr_ms / 1e3) / 1e9, 1),
        "csr_baseline_spmv_gbps": round(spmv_bytes / (csr_ms / 1e3) / 1e9, 1),
        "roofline": roofline,
        "attainable": attainable,
        "rwr_batched": rwr,
        "kernels": kernels,
        "rmat20_drivers": drivers,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
