"""A seeded sweep over random matrices and build options: for each case the
GPU format must equal the reference builder's bit for bit, and SpMV and SpMM
must meet the per-entry bound against the FP64 oracle.  The cases are drawn
once from a fixed seed, so the sweep is the same on every run."""
import os
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import ref_format as rf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # these tests need a GPU
    pytest.skip("no GPU", allow_module_level=True)

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from paper_1103_2405_amd import TiledMatrix  # noqa: E402
from test_gpu_parity import assert_same_format  # noqa: E402

TOL = 1e-5


def _cases(n_cases=32, seed=2405):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_cases):
        square = rng.random() < 0.7
        n_rows = int(rng.integers(1, 1500))
        n_cols = n_rows if square else int(rng.integers(1, 1500))
        density = float(rng.choice([0.002, 0.01, 0.03]))
        power = float(rng.choice([0.0, 0.8, 1.2]))
        W = int(rng.choice([0, 16, 100, 512]))            # 0: one tile
        wl = None if rng.random() < 0.3 else int(rng.choice([4, 64, 300, 2048]))
        split = int(rng.choice([-1, 0, 8, 64]))
        pad = bool(rng.random() < 0.2)
        out.append((i, n_rows, n_cols, density, power, W, wl, split, pad))
    return out


def _bounded(y, ref, bound):
    bad = np.flatnonzero(np.abs(y - ref) > bound)
    assert bad.size == 0, (bad[:10], np.abs(y - ref)[bad[:10]], bound[bad[:10]])


@pytest.mark.parametrize("i,n_rows,n_cols,density,power,W,wl,split,pad", _cases())
def test_random_case(i, n_rows, n_cols, density, power, W, wl, split, pad):
    csr = gg.random_csr(n_rows, n_cols, density, 500 + i, power=power if power > 0 else None)
    print("case", i, n_rows, n_cols, len(csr[3]), "W", W, "wl", wl, "split", split, "pad", pad, flush=True)
    gm = TiledMatrix(csr, tile_width=W, wl=wl, split_len=split, camping_pad=pad, perf_table=None)
    if wl is not None:  # autotuned sizes come from the built-in table; formats are compared for given sizes
        ref = rf.build(csr, W=W if W > 0 else (1 << 23), n_tiles=-1, wl=[wl] * 4096, S=64, split_len=split,
                       camping_pad=pad, table=None, max_act_warp=8192)
        assert_same_format(gm.export_format(), ref)
    x = gg.uniform_f32(n_cols, 600 + i)
    y = gm.spmv(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    _bounded(y, oracle.spmv(csr, x), TOL * oracle.absmv(csr, x))
    for k in (3, 8):
        X = gg.uniform_f32(n_cols * k, 700 + i).reshape(n_cols, k)
        Y = gm.spmm(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
        ref_y = oracle.spmm(csr, X)
        absY = np.stack([oracle.absmv(csr, np.ascontiguousarray(X[:, q])) for q in range(k)], axis=1)
        _bounded(Y.ravel(), ref_y.ravel(), TOL * absY.ravel())
    gm.close()
