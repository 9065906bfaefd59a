"""The rocprofv3 summary helpers on small hand-made CSV files: kernel
statistics ordering, traffic scaled by the copy kernel's reading, per-dispatch
counter means, and the source hash that invalidates a stale traffic figure."""
import csv
import os

import pytest

from paper_1103_2405_amd import profsum


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _counter_run(d, counter, rows):
    _write(os.path.join(d, "host", "run_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [(k, counter, v) for k, v in rows])


def test_stats_sorted_by_total_time(tmp_path):
    _write(str(tmp_path / "r" / "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [("small", 10, 1000, 100, 1.0), ("big", 2, 90000, 45000, 90.0), ("mid", 3, 9000, 3000, 9.0)])
    text = profsum.summarize_stats(str(tmp_path / "r"), "cmd here")
    body = [ln.split()[0] for ln in text.splitlines() if not ln.startswith("#")][1:]
    assert body == ["big", "mid", "small"]
    assert "# command: cmd here" in text


def test_counters_scaled_by_copy_and_hash_checked(tmp_path, monkeypatch):
    # the copy of 1 MiB reads 512 KiB on FETCH_SIZE (scale 2) and 1024 KiB on WRITE_SIZE (scale 1)
    _counter_run(str(tmp_path / "f"), "FETCH_SIZE", [("k_tile_spmv_pr", 100.0), ("k_tile_spmv_pr", 300.0),
                                                    ("__amd_rocclr_copyBuffer", 512.0), ("other", 7.0)])
    _counter_run(str(tmp_path / "w"), "WRITE_SIZE", [("k_tile_spmv_pr", 10.0), ("k_tile_spmv_pr", 30.0),
                                                    ("__amd_rocclr_copyBuffer", 1024.0)])
    text = profsum.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), "^k_tile_spmv", 1 << 20, "c")
    kv = dict(ln.split(": ", 1) for ln in text.splitlines() if ": " in ln and not ln.startswith("#"))
    assert int(kv["dispatches"]) == 2
    assert int(kv["traffic_bytes_per_launch"]) == (200 * 2 + 20 * 1) * 1024
    out = tmp_path / "t.txt"
    out.write_text(text)
    assert profsum.read_traffic(str(out)) == (200 * 2 + 20) * 1024
    monkeypatch.setattr(profsum, "source_hash", lambda: "changed")
    assert profsum.read_traffic(str(out)) is None
    assert profsum.read_traffic(str(tmp_path / "missing.txt")) is None


def test_counters_need_the_copy_kernel(tmp_path):
    _counter_run(str(tmp_path / "f"), "FETCH_SIZE", [("k_tile_spmv", 1.0)])
    _counter_run(str(tmp_path / "w"), "WRITE_SIZE", [("k_tile_spmv", 1.0)])
    with pytest.raises(SystemExit):
        profsum.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), "^k_tile_spmv", 1024, "c")


def test_pmc_means_over_several_runs(tmp_path):
    _counter_run(str(tmp_path / "a"), "TCC_HIT_sum", [("k_tile_spmv_pr", 4.0), ("k_tile_spmv", 8.0), ("x", 100.0)])
    _counter_run(str(tmp_path / "b"), "TCC_MISS_sum", [("k_tile_spmv_pr", 1.0), ("k_tile_spmv_pr", 2.0)])
    text = profsum.summarize_pmc([str(tmp_path / "a"), str(tmp_path / "b")], "^k_tile_spmv", "c")
    assert "TCC_HIT_sum: 6.0  (2 dispatches)" in text
    assert "TCC_MISS_sum: 1.5  (2 dispatches)" in text
    with pytest.raises(SystemExit):
        profsum.summarize_pmc([str(tmp_path / "a")], "^nothing", "c")
