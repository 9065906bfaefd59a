"""Reference implementation of the paper's parameter tuning (Section 3.3,
Appendix E, Algorithms 1-3, Eq. 1-5).  TEST INFRASTRUCTURE ONLY.

Algorithm 1 (number of tiles): add tiles of TILE_WIDTH columns of the
column-sorted matrix while the first column of the next tile holds at least
two entries.

Algorithm 2 (workload size of one tile): candidates run from the length of the
tile's first row (lower bound) to the tile's nnz divided by the number of
resident wavefronts (upper bound), in steps of the first row's length; the
candidate whose modelled time is strictly smallest wins (so ties keep the
smaller size).  If the upper bound is below the lower bound the lower bound is
used.

Algorithm 3 (performance model of a tile for one workload size): partition the
tile exactly as the packer does, assign workload j to round j // MAX_ACT_WARP
(Eq. 1), and for every round add the padded area (Eq. 4) and the table
throughput of the padded shape (Eq. 5); the round's time is its area divided by
its mean throughput (Eq. 3) and the tile's time is the sum over rounds (Eq. 2).

Readings where the paper is silent (each also listed in the design notes):
  * heavy rows longer than split_len are cut into chunks of split_len entries
    (one-row row-major workloads) and do not take part in the WL bounds; the
    lower bound is the first row that is not split.  With the automatic rule a
    tile's split length is its nnz divided by the number of resident
    wavefronts, rounded up to a multiple of S and kept in [S, 8192]
    (`tile_split_len`), so that no row is longer than one wavefront's share;
  * h = max(1, floor(WL / w)); a column-major workload then takes
    ceil(h / S) * S real rows when that many remain;
  * the throughput table is a full grid over powers of two of w and h; a shape
    is looked up at the nearest power of two of each side in log scale (ties
    round up), clamped to the grid;
  * the model is evaluated in double precision in exactly this order of
    operations: per round, mean = sum_perf / count, then time += area / mean.

The partition routine here is the one the reference format builder uses.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

RM, CM = 0, 1


def ceil_to(v: int, s: int) -> int:
    return -(-v // s) * s


def rm_pad(w: int, S: int) -> int:
    """Padded row length of a row-major workload (Solution 3: rows padded to a
    multiple of the warp size).  With S = 64 rows of at most 32 entries pad to
    32, the paper's own warp size."""
    return S // 2 if S >= 64 and 2 * w <= S else ceil_to(w, S)


def partition_rows(lengths: Sequence[int], wl: int, S: int, split_len: int) -> List[Tuple]:
    """Greedy packing of a tile's rows (sorted by decreasing length) into
    workloads (Solution 3, Algorithm 3 lines 7-16).

    Returns tuples (layout, w, w_pad, h_pad, row_begin, n_rows, chunk, n_chunks)
    in emission order; chunk >= 0 marks one chunk of a split heavy row, whose
    w is the chunk's length.
    """
    out = []
    R = len(lengths)
    i = 0
    while i < R:
        w = int(lengths[i])
        if split_len > 0 and w > split_len:
            nch = -(-w // split_len)
            for k in range(nch):
                cw = min(split_len, w - k * split_len)
                out.append((RM, cw, ceil_to(cw, S), 1, i, 1, k, nch))
            i += 1
            continue
        h = min(max(1, wl // w), R - i)
        if w >= h:
            out.append((RM, w, rm_pad(w, S), h, i, h, -1, 0))
            i += h
        else:
            hp = ceil_to(h, S)
            nr = min(hp, R - i)
            out.append((CM, w, w, hp, i, nr, -1, 0))
            i += nr
    return out


def nearest_log2(v: int) -> int:
    """Nearest power-of-two exponent of v >= 1 in log scale; ties round up."""
    k = int(v).bit_length() - 1
    return k + 1 if v * v >= (1 << (2 * k + 1)) else k


class PerfTable:
    """Throughput table over a grid of powers of two: value[kind][lw][lh]."""

    def __init__(self, dense: np.ndarray, sparse: np.ndarray):
        self.grid = {"dense": np.asarray(dense, np.int64), "sparse": np.asarray(sparse, np.int64)}

    @staticmethod
    def load(path: str) -> "PerfTable":
        entries: Dict[str, Dict[Tuple[int, int], int]] = {"dense": {}, "sparse": {}}
        with open(path) as f:
            for line in f:
                line = line.split("#", 1)[0].strip()
                if not line:
                    continue
                kind, lw, lh, v = line.split()
                entries[kind][(int(lw), int(lh))] = int(v)
        grids = []
        for kind in ("dense", "sparse"):
            e = entries[kind]
            nw = max(k[0] for k in e) + 1
            nh = max(k[1] for k in e) + 1
            g = np.zeros((nw, nh), np.int64)
            for (a, b), v in e.items():
                g[a, b] = v
            grids.append(g)
        return PerfTable(*grids)

    def perf(self, kind: str, w: int, h: int) -> int:
        g = self.grid[kind]
        lw = min(nearest_log2(w), g.shape[0] - 1)
        lh = min(nearest_log2(h), g.shape[1] - 1)
        return int(g[lw, lh])


def shape_of(wl: Tuple) -> Tuple[int, int]:
    """Padded (w, h) of a workload as the model sees it."""
    layout, w, w_pad, h_pad = wl[0], wl[1], wl[2], wl[3]
    return (w_pad, h_pad)


def model_time(lengths: Sequence[int], wl: int, table: PerfTable, kind: str,
               max_act_warp: int, S: int, split_len: int) -> float:
    """Algorithm 3 / Eq. 1-5: modelled time of one tile at workload size wl."""
    wls = partition_rows(lengths, wl, S, split_len)
    n_iter = -(-len(wls) // max_act_warp)
    P = [0.0] * n_iter
    Size = [0.0] * n_iter
    Cnt = [0] * n_iter
    for j, w in enumerate(wls):
        it = j // max_act_warp
        pw, ph = shape_of(w)
        P[it] += float(table.perf(kind, pw, ph))
        Size[it] += float(pw * ph)
        Cnt[it] += 1
    total = 0.0
    for i in range(n_iter):
        mean = P[i] / float(Cnt[i])
        total += Size[i] / mean
    return total


def choose_wl(lengths: Sequence[int], tile_nnz: int, table: PerfTable, kind: str,
              max_act_warp: int, S: int, split_len: int) -> int:
    """Algorithm 2: workload size with the least modelled time."""
    first = None
    for L in lengths:
        if not (split_len > 0 and L > split_len):
            first = int(L)
            break
    if first is None:  # every row is split: the size only bounds nothing
        return split_len if split_len > 0 else (int(lengths[0]) if len(lengths) else 1)
    low = first
    up = tile_nnz // max_act_warp
    if up < low:
        return low
    best_t = math.inf
    best = 0
    wl = low
    while wl <= up:
        t = model_time(lengths, wl, table, kind, max_act_warp, S, split_len)
        if t < best_t:
            best_t = t
            best = wl
        wl += low
    return best


SPLIT_CAP = 8192


def tile_split_len(split_len: int, tile_nnz: int, max_act_warp: int, S: int) -> int:
    """Split length used for one tile: -1 = automatic (per-wavefront share of
    the tile, rounded up to a multiple of S, within [S, 8192]); 0 = no split;
    otherwise the given length."""
    if split_len >= 0:
        return split_len
    share = -(-tile_nnz // max_act_warp)
    return min(SPLIT_CAP, max(S, ceil_to(share, S)))


def count_tiles(clen_sorted: np.ndarray, W: int) -> int:
    """Algorithm 1: dense tiles while the first column of the next tile has >= 2 entries."""
    n_cols = len(clen_sorted)
    NT = -(-n_cols // W)
    T = 0
    while T < NT and clen_sorted[T * W] >= 2:
        T += 1
    return T
