"""The builder's host work (Algorithm 3's partition of every tile, the
descriptors, the pipelined pack) runs on a pool of host threads; the format
must not depend on how many.  A child process built with TC_HOST_THREADS=1
(every loop on the calling thread) writes its format; this process, with the
default pool, builds the same matrices and compares them bit for bit."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # these tests need a GPU
    pytest.skip("no GPU", allow_module_level=True)

import graphgen as gg  # noqa: E402
from paper_1103_2405_amd import TiledMatrix  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CASES = [dict(panels=-1), dict(tile_width=256, split_len=256), dict(tile_width=32, n_tiles=1500, split_len=-1, wl=300)]
# tiles at least: 64 (the host pool takes loops of 64 tiles or more), 1024 (the
# pack in four batches)
MIN_TILES = [64, 64, 1024]
KEYS = ["tile_nnz", "tile_wl", "tile_row_off", "rows_sorted", "rows_len", "wl_tile", "wl_layout", "wl_w", "wl_w_pad",
        "wl_h_pad", "wl_row_begin", "wl_n_rows", "wl_chunk", "wl_n_chunks", "wl_data_off", "wl_rowid_off", "idx",
        "val", "rowid"]

CHILD = r'''
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import graphgen as gg
from paper_1103_2405_amd import TiledMatrix
from tests.test_gpu_host_threads import CASES, KEYS, matrix
out = {}
for i, kw in enumerate(CASES):
    tm = TiledMatrix(matrix(), **kw)
    f = tm.export_format()
    for k in KEYS:
        out["%d_%s" % (i, k)] = np.asarray(f[k])
    tm.close()
np.savez(sys.argv[2], **out)
print("child ok", flush=True)
'''


def matrix():
    return gg.pagerank_matrix(gg.rmat(16, 16, seed=16))


def test_format_independent_of_host_threads(tmp_path):
    path = str(tmp_path / "one_thread.npz")
    env = dict(os.environ, TC_HOST_THREADS="1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, path], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    one = np.load(path)
    for i, kw in enumerate(CASES):
        tm = TiledMatrix(matrix(), **kw)
        f = tm.export_format()
        assert f["n_tiles_total"] >= MIN_TILES[i], (kw, f["n_tiles_total"])
        for k in KEYS:
            a, b = np.asarray(f[k]), one["%d_%s" % (i, k)]
            assert a.shape == b.shape and np.array_equal(a.view(np.uint8), b.view(np.uint8)), (kw, k)
        tm.close()
