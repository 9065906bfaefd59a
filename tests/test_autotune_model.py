"""Pins of the reference tuning (Algorithms 1-3, Eq. 1-5) on cases whose
answer follows by hand."""
import numpy as np

from oracle.autotune import (CM, RM, PerfTable, choose_wl, count_tiles, model_time, nearest_log2,
                             partition_rows)


def const_table(v=100):
    g = np.full((16, 16), v, np.int64)
    return PerfTable(g, g)


def test_algorithm1_tile_count():
    assert count_tiles(np.array([5, 5, 3, 2, 1, 1, 1]), 2) == 2
    assert count_tiles(np.array([5, 5, 3, 2, 1, 1, 1]), 3) == 2
    assert count_tiles(np.array([1, 1, 1]), 1) == 0
    # the loop bound is the number of (possibly partial) tiles: 5 columns of
    # length 4 at width 4 give 2 tiles, the second one column wide
    assert count_tiles(np.array([4, 4, 4, 4, 4]), 4) == 2


def test_partition_figure1():
    assert partition_rows([2, 2, 2, 2, 1, 1, 1, 1], 4, 2, 0) == [
        (RM, 2, 2, 2, 0, 2, -1, 0), (RM, 2, 2, 2, 2, 2, -1, 0), (CM, 1, 1, 4, 4, 4, -1, 0)]


def test_partition_column_major_fills_padded_rows():
    # w=1, WL=3 -> h=3 padded to 4 real rows when 4 remain (S = 4)
    assert partition_rows([1] * 6, 3, 4, 0) == [(CM, 1, 1, 4, 0, 4, -1, 0), (CM, 1, 1, 4, 4, 2, -1, 0)]


def test_partition_split_rows():
    assert partition_rows([10, 3], 6, 4, 4) == [
        (RM, 4, 4, 1, 0, 1, 0, 3), (RM, 4, 4, 1, 0, 1, 1, 3), (RM, 2, 4, 1, 0, 1, 2, 3),
        (RM, 3, 4, 1, 1, 1, -1, 0)]


def test_model_constant_table_is_padded_area():
    # 640 rows of length 3, S = 64: WL 3..9 gives row-major rows padded to
    # 32 (rows of at most half a wavefront: 32 * 640 padded area); S = 128
    # pads them to 128; WL >= 12 gives column-major blocks of 64 rows with no
    # padding (3 * 640).
    L = [3] * 640
    t = const_table(100)
    assert model_time(L, 3, t, "dense", 10 ** 6, 64, 0) == 32 * 640 / 100
    assert model_time(L, 3, t, "dense", 10 ** 6, 128, 0) == 64 * 640 / 100
    # rows of 33 entries are longer than half a wavefront: padded to 64
    assert model_time([33] * 64, 33, t, "dense", 10 ** 6, 64, 0) == 64 * 64 / 100
    assert model_time(L, 12, t, "dense", 10 ** 6, 64, 0) == 3 * 640 / 100
    # Algorithm 2 picks the first size without padding (ties keep the smaller)
    assert choose_wl(L, 1920, t, "dense", 100, 64, 0) == 12


def test_model_rounds_eq1_to_eq5():
    # three workloads of shapes (64 x 1), (64 x 1), (64 x 2); two per round
    g = np.full((16, 16), 10, np.int64)
    g[6, 0] = 20   # w = 64, h = 1
    g[6, 1] = 40   # w = 64, h = 2
    t = PerfTable(g, g)
    L = [64, 64, 64, 64]
    # WL = 64: four one-row workloads; rounds of 2: (64+64)/20 * 2
    assert model_time(L, 64, t, "dense", 2, 64, 0) == 2 * (128 / 20)
    # WL = 128: two workloads of 2 rows in one round: 256 / 40
    assert model_time(L, 128, t, "dense", 2, 64, 0) == 256 / 40
    # Algorithm 2 with upper bound 256 // 2 = 128 compares 64 and 128
    assert choose_wl(L, 256, t, "dense", 2, 64, 0) == 128


def test_choose_wl_bounds():
    t = const_table()
    # upper bound below the lower bound -> lower bound
    assert choose_wl([50, 10], 60, t, "dense", 8192, 64, 0) == 50
    # split rows do not set the lower bound
    assert choose_wl([100000, 7, 7], 100014, t, "dense", 8192, 64, 8192) == 7


def test_nearest_log2():
    assert [nearest_log2(v) for v in (1, 2, 3, 5, 6, 11, 12, 64, 90, 91)] == [0, 1, 2, 2, 3, 3, 4, 6, 6, 7]


def test_tile_split_len_by_hand():
    from oracle.autotune import tile_split_len
    # given lengths are used as they are (0: never split, the paper's rule)
    assert tile_split_len(0, 10 ** 9, 8192, 64) == 0
    assert tile_split_len(777, 10, 8192, 64) == 777
    # automatic: the tile's entries per resident wavefront, rounded up to a
    # multiple of S, kept within [S, 8192]
    assert tile_split_len(-1, 8192 * 100 + 1, 8192, 64) == 128      # ceil(100.0001) = 101 -> 128
    assert tile_split_len(-1, 8192 * 128, 8192, 64) == 128          # exactly 128 per wavefront
    assert tile_split_len(-1, 8192 * 128 + 1, 8192, 64) == 192      # 129 -> 192
    assert tile_split_len(-1, 5, 8192, 64) == 64                    # below one wave width: S
    assert tile_split_len(-1, 0, 8192, 64) == 64                    # empty tile: S
    assert tile_split_len(-1, 1 << 27, 8192, 64) == 8192            # 16384 capped at 8192
    assert tile_split_len(-1, 1000, 10, 4) == 100                   # other S and wavefront counts
    assert tile_split_len(-1, 1001, 10, 4) == 104


def test_perf_table_lookup_rounds_and_clamps():
    # value = 100 lw + lh on a 4 x 3 grid makes every lookup's cell visible
    g = np.array([[100 * a + b for b in range(3)] for a in range(4)], np.int64)
    t = PerfTable(g, 2 * g)
    assert t.perf("dense", 1, 1) == 0
    assert t.perf("dense", 2, 4) == 102
    assert t.perf("dense", 3, 3) == 202        # 3 rounds up to 4 in log scale
    assert t.perf("dense", 5, 1) == 200        # 5 rounds down to 4
    assert t.perf("dense", 6, 1) == 300        # 6 rounds up to 8
    assert t.perf("dense", 1000, 1) == 300     # past the grid: the last column
    assert t.perf("dense", 8, 4096) == 302     # past the grid in h as well
    assert t.perf("sparse", 1000, 4096) == 604  # the sparse grid, clamped the same way
