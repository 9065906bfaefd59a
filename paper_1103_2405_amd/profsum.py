"""Summaries of rocprofv3 output as short text files for profiles/.

Three kinds:

* ``stats``: the kernel-trace statistics (rocprofv3 --kernel-trace --stats) of
  one run, the kernels sorted by total time, with calls and mean duration.
* ``counters``: HBM traffic of one kernel from two counter passes
  (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, both in KiB per
  dispatch).  Each counter is scaled by what it reads for a plain device copy
  of known size in the same run (the copy reads and writes ``--copy-bytes``),
  so the figures are bytes that really crossed the L2/fabric boundary.  The
  file records a hash of the library sources; bench.py reports the traffic
  only while the kernels are unchanged.
* ``pmc``: the mean per dispatch of every counter collected for one kernel in
  one or more counter runs (cache hits and misses, requests to the fabric).

    python -m paper_1103_2405_amd.profsum stats RUN_DIR --cmd "..." --out FILE
    python -m paper_1103_2405_amd.profsum counters FETCH_DIR WRITE_DIR --kernel REGEX \\
        --copy-bytes N --cmd "..." --out FILE
    python -m paper_1103_2405_amd.profsum pmc RUN_DIR [RUN_DIR ...] --kernel REGEX --cmd "..." --out FILE
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_KERNEL = "copyBuffer"


def source_hash() -> str:
    """SHA-256 over the library sources (names and contents, sorted)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*"))):
        if os.path.isfile(p):
            h.update(os.path.basename(p).encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise SystemExit("no file matches " + pattern)
    return hits[0]


def summarize_stats(run_dir: str, cmd: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(_one(os.path.join(run_dir, "**", "*kernel_stats.csv")))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel statistics", "# command: " + cmd, "#",
             "%-48s %8s %14s %12s %7s" % ("kernel", "calls", "total_ms", "mean_us", "pct")]
    for r in rows[:top]:
        lines.append("%-48s %8d %14.3f %12.2f %7.2f" % (
            r["Name"][:48], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(lines) + "\n"


def _per_dispatch(run_dir: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    out = {}
    for r in csv.DictReader(open(_one(os.path.join(run_dir, "**", "*counter_collection.csv")))):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _largest_copy(d) -> float:
    vals = [v for k, vs in d.items() if COPY_KERNEL in k for v in vs]
    if not vals:
        raise SystemExit("no copy kernel in the counter run (run bench.py with --probe-copy)")
    return max(vals)


def summarize_counters(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int, cmd: str) -> str:
    rx = re.compile(kernel)
    fetch = _per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _per_dispatch(write_dir, "WRITE_SIZE")
    fk = [v for k, vs in fetch.items() if rx.search(k) for v in vs]
    wk = [v for k, vs in write.items() if rx.search(k) for v in vs]
    if not fk or not wk:
        raise SystemExit("kernel %r not found in the counter runs" % kernel)
    copy_kib = copy_bytes / 1024.0
    f_scale = copy_kib / _largest_copy(fetch)
    w_scale = copy_kib / _largest_copy(write)
    f_mean = sum(fk) / len(fk)
    w_mean = sum(wk) / len(wk)
    traffic = (f_mean * f_scale + w_mean * w_scale) * 1024.0
    lines = [
        "# HBM traffic of one kernel from rocprofv3 counter passes",
        "# command: " + cmd,
        "# FETCH_SIZE and WRITE_SIZE are KiB per dispatch; each is scaled by the",
        "# reading of the same counter for a plain device copy of copy_bytes bytes.",
        "kernel: " + kernel,
        "source_sha256: " + source_hash(),
        "dispatches: %d" % len(fk),
        "fetch_kib_per_dispatch: %.1f" % f_mean,
        "write_kib_per_dispatch: %.1f" % w_mean,
        "copy_bytes: %d" % copy_bytes,
        "fetch_scale: %.4f" % f_scale,
        "write_scale: %.4f" % w_scale,
        "traffic_bytes_per_launch: %d" % int(round(traffic)),
    ]
    return "\n".join(lines) + "\n"


def summarize_pmc(run_dirs, kernel: str, cmd: str) -> str:
    rx = re.compile(kernel)
    means, n_disp = {}, {}
    for d in run_dirs:
        for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
            if not rx.search(r["Kernel_Name"]):
                continue
            c = r["Counter_Name"]
            means[c] = means.get(c, 0.0) + float(r["Counter_Value"])
            n_disp[c] = n_disp.get(c, 0) + 1
    if not means:
        raise SystemExit("kernel %r not found in the counter runs" % kernel)
    lines = ["# rocprofv3 counters of one kernel, mean per dispatch",
             "# command: " + cmd,
             "kernel: " + kernel,
             "source_sha256: " + source_hash()]
    for c in sorted(means):
        lines.append("%s: %.1f  (%d dispatches)" % (c, means[c] / n_disp[c], n_disp[c]))
    return "\n".join(lines) + "\n"


def read_traffic(path: str):
    """traffic_bytes_per_launch from a counters summary, or None when the file
    is missing or the library sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return None
    try:
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("run_dir")
    s.add_argument("--cmd", required=True)
    s.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--out", required=True)
    m = sub.add_parser("pmc")
    m.add_argument("run_dirs", nargs="+")
    m.add_argument("--kernel", required=True)
    m.add_argument("--cmd", required=True)
    m.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.what == "stats":
        text = summarize_stats(a.run_dir, a.cmd)
    elif a.what == "counters":
        text = summarize_counters(a.fetch_dir, a.write_dir, a.kernel, a.copy_bytes, a.cmd)
    else:
        text = summarize_pmc(a.run_dirs, a.kernel, a.cmd)
    with open(a.out, "w") as f:
        f.write(text)
    print(text, end="")


if __name__ == "__main__":
    sys.exit(main())
