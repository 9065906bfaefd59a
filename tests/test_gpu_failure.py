"""Failure handling through the C ABI, forced from the host: an injected
allocator that runs out (TC_ENOMEM, every block handed back), an allocator
that works (the product still matches the oracle), and arguments of the wrong
dtype, device or length rejected by the binding before any library call."""
import ctypes
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # these tests need a GPU
    pytest.skip("no GPU", allow_module_level=True)

from paper_1103_2405_amd import TiledMatrix, DeviceCsr, csr_spmv  # noqa: E402
from paper_1103_2405_amd import tc as tcmod  # noqa: E402

ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class TorchAllocator:
    """Device blocks from torch's caching allocator; fails once `budget`
    allocations have been handed out (budget None: never)."""

    def __init__(self, budget=None):
        self.budget = budget
        self.live = {}
        self.calls = 0
        self.c_alloc = ALLOC(self._alloc)
        self.c_free = FREE(self._free)

    def _alloc(self, nbytes, ctx):
        self.calls += 1
        if self.budget is not None and self.calls > self.budget:
            return None
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, p, ctx):
        self.live.pop(p, None)


def build_with(csr, alloc):
    lib = tcmod.load_library()
    A = DeviceCsr(csr)
    o = tcmod.CBuildOpts()
    lib.tc_build_opts_default(ctypes.byref(o))
    o.tile_width, o.split_len = 1024, 256
    o.alloc = ctypes.cast(alloc.c_alloc, ctypes.c_void_p)
    o.free = ctypes.cast(alloc.c_free, ctypes.c_void_p)
    h = ctypes.c_void_p()
    c = A.c()
    st = lib.tc_build_tiled(ctypes.byref(c), ctypes.byref(o), tcmod._stream(), ctypes.byref(h))
    return st, h, A


def test_allocator_running_out_gives_enomem():
    g = gg.rmat(11, 16, seed=3)
    csr = gg.pagerank_matrix(g)
    full = TorchAllocator(None)
    st, h, _ = build_with(csr, full)
    assert st == tcmod.TC_OK
    n_alloc = full.calls
    tcmod.load_library().tc_destroy(h)
    assert n_alloc >= 4 and not full.live
    for budget in sorted({0, 1, n_alloc // 2, n_alloc - 1}):
        al = TorchAllocator(budget)
        say("injected allocator: %d of %d allocations succeed" % (budget, n_alloc))
        st, h, _ = build_with(csr, al)
        assert st == tcmod.TC_ENOMEM, st
        assert b"allocator callback returned NULL" in tcmod.load_library().tc_last_error()
        assert not h.value
        assert al.calls == budget + 1
        assert not al.live, "blocks of the failed build were not handed back"


def test_working_allocator_holds_every_buffer():
    g = gg.rmat(11, 16, seed=3)
    csr = gg.pagerank_matrix(g)
    al = TorchAllocator(None)
    st, h, A = build_with(csr, al)
    assert st == tcmod.TC_OK, tcmod.load_library().tc_last_error()
    assert al.live
    lib = tcmod.load_library()
    x = gg.uniform_f32(g.n, 101)
    xt = torch.from_numpy(x).cuda()
    y = torch.empty(g.n, dtype=torch.float32, device="cuda")
    assert lib.tc_spmv(h, tcmod._ptr(xt), tcmod._ptr(y), tcmod._stream()) == tcmod.TC_OK
    yy = y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(yy - oracle.spmv(csr, x)) <= 1e-5 * oracle.absmv(csr, x))
    lib.tc_destroy(h)
    assert not al.live, "destroy did not hand every block back"


def test_binding_rejects_bad_vectors_before_any_call():
    g = gg.rmat(9, 8, seed=4)
    csr = gg.pagerank_matrix(g)
    n = g.n
    with TiledMatrix(csr, tile_width=256) as A:
        good = torch.rand(n, device="cuda")
        for bad in (torch.rand(n, device="cuda", dtype=torch.float64),  # wrong dtype
                    torch.rand(n),                                      # host memory
                    torch.rand(n - 1, device="cuda"),                   # too short
                    torch.rand(n + 1, device="cuda"),                   # too long
                    torch.rand(2 * n, device="cuda")[::2]):             # not contiguous
            with pytest.raises(ValueError):
                A.spmv(bad)
            with pytest.raises(ValueError):
                A.spmv(good, bad)
            with pytest.raises(ValueError):
                A.spmv_internal(bad, torch.empty(n, device="cuda"))
            with pytest.raises(ValueError):
                csr_spmv(DeviceCsr(csr), bad)
        for X in (torch.rand(n, 4, device="cuda", dtype=torch.float64), torch.rand(n - 1, 4, device="cuda"),
                  torch.rand(n, 4), torch.rand(4, n, device="cuda").t(), torch.rand(n, device="cuda")):
            with pytest.raises(ValueError):
                A.spmm(X)
        with pytest.raises(ValueError):
            A.spmm(torch.rand(n, 4, device="cuda"), torch.empty(n, 5, device="cuda"))
        with pytest.raises(ValueError):
            A.pagerank(out=torch.empty(n - 1, device="cuda"))
        # the good vectors still work
        y = A.spmv(good)
        assert y.shape == (n,)
