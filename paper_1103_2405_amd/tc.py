"""Python binding of libtcspmv (include/tcspmv.h): argument marshalling only.

Device memory and streams come from PyTorch; every computation runs in the
library's HIP kernels.  If the library is missing or cannot be loaded, every
call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcspmv.so")
DEFAULT_PERF_TABLE = os.path.join(_HERE, "data", "perf_table_gfx950.txt")

TC_OK, TC_EINVAL, TC_ENOMEM, TC_EHIP, TC_ENOTCONV, TC_EUNSUPPORTED = range(6)
_STATUS = {1: "TC_EINVAL", 2: "TC_ENOMEM", 3: "TC_EHIP", 4: "TC_ENOTCONV", 5: "TC_EUNSUPPORTED"}


class TcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class NotConverged(TcError):
    pass


vp = ctypes.c_void_p
i32, i64 = ctypes.c_int32, ctypes.c_int64


class CCsr(ctypes.Structure):
    _fields_ = [("n_rows", i64), ("n_cols", i64), ("nnz", i64),
                ("row_ptr", vp), ("col_idx", vp), ("val", vp)]


class CBuildOpts(ctypes.Structure):
    _fields_ = [("tile_width", i32), ("n_tiles", i32), ("wl_policy", i32), ("wl_all", i32),
                ("wl_per_tile", vp), ("n_wl_per_tile", i32), ("wave", i32), ("split_len", i32),
                ("camping_pad", i32), ("relabel", i32), ("max_act_warp", i32), ("xcd_groups", i32), ("kernel", i32),
                ("value_map", i32), ("slices", i32), ("tile_bounds", vp), ("n_tile_bounds", i32),
                ("lds_stage", i32), ("panels", i32), ("panel_rows", i32), ("panel_waves", i32),
                ("perf_table", ctypes.c_char_p), ("alloc", vp), ("free", vp), ("alloc_ctx", vp)]


class CInfo(ctypes.Structure):
    _fields_ = [("n_rows", i64), ("n_cols", i64), ("nnz", i64),
                ("tile_width", i32), ("wave", i32), ("split_len", i32), ("relabel", i32),
                ("xcd_groups", i32), ("kernel", i32), ("n_dense_tiles", i32), ("n_tiles", i32),
                ("n_workloads", i64), ("nnz_pad", i64), ("n_rowid", i64), ("n_rows_sorted", i64),
                ("n_split_rows", i64), ("n_partials", i64), ("n_dangling", i64), ("device_bytes", i64),
                ("build_us", ctypes.c_double), ("model_us", ctypes.c_double),
                ("n_panels", i32), ("n_col_tiles", i32), ("panel_rows", i32), ("panel_waves", i32)]


_VIEW_FIELDS = [("cperm", np.int32, "n_cols"), ("rowmap", np.int32, "n_rows"),
                ("tile_col_begin", np.int64, "n_tiles"), ("tile_col_end", np.int64, "n_tiles"),
                ("tile_nnz", np.int64, "n_tiles"), ("tile_wl", np.int64, "n_tiles"),
                ("tile_split", np.int64, "n_tiles"),
                ("tile_row_off", np.int64, "n_tiles+1"), ("rows_sorted", np.int32, "n_rows_sorted"),
                ("rows_len", np.int32, "n_rows_sorted"),
                ("wl_tile", np.int32, "n_workloads"), ("wl_layout", np.int32, "n_workloads"),
                ("wl_w", np.int32, "n_workloads"), ("wl_w_pad", np.int32, "n_workloads"),
                ("wl_h_pad", np.int32, "n_workloads"), ("wl_row_begin", np.int32, "n_workloads"),
                ("wl_n_rows", np.int32, "n_workloads"), ("wl_chunk", np.int32, "n_workloads"),
                ("wl_n_chunks", np.int32, "n_workloads"), ("wl_data_off", np.int64, "n_workloads"),
                ("wl_rowid_off", np.int64, "n_workloads"), ("idx", np.int32, "nnz_pad"),
                ("val", np.float32, "nnz_pad"), ("rowid", np.int32, "n_rowid"),
                ("coo_row", np.int32, "nnz_coo"), ("coo_col", np.int32, "nnz_coo"),
                ("coo_val", np.float32, "nnz_coo"), ("panel_begin", np.int64, "n_panels+1")]


class CFormatView(ctypes.Structure):
    _fields_ = [(name, vp) for name, _, _ in _VIEW_FIELDS]


class CTiming(ctypes.Structure):
    _fields_ = [("tile_kernel_ms", ctypes.c_double), ("tile_launches", i64), ("spmv_calls", i64)]


EXPORTED = ["tc_build_opts_default", "tc_build_tiled", "tc_spmv", "tc_spmv_internal", "tc_spmv_tiles", "tc_spmm",
            "tc_pagerank", "tc_hits", "tc_rwr", "tc_csr_spmv", "tc_handle_info", "tc_export_format",
            "tc_set_timing", "tc_get_timing", "tc_destroy", "tc_last_error", "tc_release_cached_memory",
            "tc_rwr_multi", "tc_csr_transpose", "tc_rwr_edge_weights", "tc_rwr_iterates", "tc_rwr_adjoint",
            "tc_rwr_theta_grad", "tc_gather_rows", "tc_refresh_values", "tc_stream_read", "tc_gather_read",
            "tc_spmm_internal_noalloc"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtcspmv.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libtcspmv.so is not built (%s); run python -m paper_1103_2405_amd.build" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.tc_build_opts_default.argtypes = [P(CBuildOpts)]
    lib.tc_build_opts_default.restype = None
    lib.tc_build_tiled.argtypes = [P(CCsr), P(CBuildOpts), vp, P(vp)]
    lib.tc_spmv.argtypes = [vp, vp, vp, vp]
    lib.tc_spmv_internal.argtypes = [vp, vp, vp, vp]
    lib.tc_spmv_tiles.argtypes = [vp, vp, vp, vp]
    lib.tc_stream_read.argtypes = [vp, i64, vp, vp]
    lib.tc_gather_read.argtypes = [vp, i64, vp, vp, i64, vp, vp]
    lib.tc_spmm_internal_noalloc.argtypes = [vp, vp, vp, i32, vp]
    lib.tc_spmm.argtypes = [vp, vp, vp, i32, vp]
    lib.tc_pagerank.argtypes = [vp, ctypes.c_float, ctypes.c_float, i32, i32, vp, P(i32), P(ctypes.c_double), vp]
    lib.tc_hits.argtypes = [vp, ctypes.c_float, i32, i32, vp, vp, P(i32), P(ctypes.c_double), vp]
    lib.tc_rwr.argtypes = [vp, vp, i32, ctypes.c_float, ctypes.c_float, i32, i32, vp, P(i32),
                           P(ctypes.c_double), vp]
    lib.tc_csr_spmv.argtypes = [P(CCsr), vp, vp, vp]
    lib.tc_rwr_multi.argtypes = [vp, i32, vp, ctypes.c_float, ctypes.c_float, i32, i32, i32, vp, P(i32), vp, vp]
    f32 = ctypes.c_float
    lib.tc_csr_transpose.argtypes = [P(CCsr), vp, vp, vp, vp, vp]
    lib.tc_gather_rows.argtypes = [vp, i64, vp, i64, i32, vp, vp]
    lib.tc_refresh_values.argtypes = [vp, vp, vp]
    lib.tc_rwr_edge_weights.argtypes = [i64, i64, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.tc_rwr_iterates.argtypes = [vp, i32, f32, i32, i32, vp, vp, vp]
    lib.tc_rwr_adjoint.argtypes = [vp, vp, vp, vp, i32, f32, i32, i32, vp, vp, vp, vp, vp]
    lib.tc_rwr_theta_grad.argtypes = [i64, i64, vp, i32, vp, vp, vp, vp, vp, f32, vp, vp]
    lib.tc_handle_info.argtypes = [vp, P(CInfo)]
    lib.tc_export_format.argtypes = [vp, P(CFormatView)]
    lib.tc_set_timing.argtypes = [vp, i32]
    lib.tc_get_timing.argtypes = [vp, P(CTiming)]
    lib.tc_destroy.argtypes = [vp]
    lib.tc_destroy.restype = None
    lib.tc_release_cached_memory.argtypes = []
    lib.tc_release_cached_memory.restype = ctypes.c_size_t
    lib.tc_last_error.argtypes = []
    lib.tc_last_error.restype = ctypes.c_char_p
    for f in EXPORTED:
        if f not in ("tc_build_opts_default", "tc_destroy", "tc_last_error", "tc_release_cached_memory"):
            getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int, what: str):
    if st != TC_OK:
        msg = (load_library().tc_last_error() or b"").decode(errors="replace")
        cls = NotConverged if st == TC_ENOTCONV else TcError
        raise cls(st, msg or what)


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t, shape, name: str) -> torch.Tensor:
    """A float32, contiguous GPU tensor of exactly `shape` (checked before any
    pointer reaches the library: a wrong dtype, device or length would make the
    kernels read or write outside the buffer)."""
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)
    if t.dtype != torch.float32:
        raise ValueError("%s must be float32, not %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape) != tuple(shape) and not (len(shape) == 1 and t.dim() == 1 and t.numel() == shape[0]):
        raise ValueError("%s must have shape %s, not %s" % (name, tuple(shape), tuple(t.shape)))
    return t


def _dev(a, dtype, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)
    return t.contiguous()


class DeviceCsr:
    """CSR arrays resident on the GPU (row_ptr int64, col int32, val float32)."""

    def __init__(self, csr, device="cuda"):
        n_rows, n_cols, rp, col, val = csr
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.row_ptr = _dev(rp, torch.int64, device)
        self.col = _dev(col, torch.int32, device)
        self.val = _dev(val, torch.float32, device)
        self.nnz = int(self.col.numel())

    def c(self) -> CCsr:
        return CCsr(self.n_rows, self.n_cols, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                    self.val.data_ptr())


def csr_spmv(A: DeviceCsr, x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Plain CSR SpMV (one thread per row) -- the baseline kernel."""
    lib = load_library()
    _need(x, (A.n_cols,), "x")
    if y is None:
        y = torch.empty(A.n_rows, dtype=torch.float32, device=x.device)
    _need(y, (A.n_rows,), "y")
    c = A.c()
    _check(lib.tc_csr_spmv(ctypes.byref(c), _ptr(x), _ptr(y), _stream(stream)), "tc_csr_spmv")
    return y


class TiledMatrix:
    """A matrix in the tiled composite format (the library handle)."""

    def __init__(self, csr, tile_width: int = 0, n_tiles: int = -1, wl: Optional[Sequence[int] | int] = None,
                 wave: int = 64, split_len: int = -1, camping_pad: bool = False, relabel: int = -1,
                 max_act_warp: int = 0, perf_table: Optional[str] = "default", xcd_groups: int = -1,
                 kernel: str = "composite", value_map: bool = False, slices: int = 0,
                 tile_bounds: Optional[Sequence[int]] = None, lds_stage: int = 0, panels: int = 0,
                 panel_rows: int = 0, panel_waves: int = 0, stream=None):
        lib = load_library()
        A = csr if isinstance(csr, DeviceCsr) else DeviceCsr(csr)
        self.n_rows, self.n_cols, self.nnz = A.n_rows, A.n_cols, A.nnz
        o = CBuildOpts()
        lib.tc_build_opts_default(ctypes.byref(o))
        o.tile_width, o.n_tiles, o.wave, o.split_len = tile_width, n_tiles, wave, split_len
        o.camping_pad, o.relabel, o.max_act_warp = int(camping_pad), relabel, max_act_warp
        if xcd_groups >= 0:
            o.xcd_groups = xcd_groups
        if kernel not in ("composite", "coo"):
            raise ValueError("kernel must be 'composite' or 'coo'")
        o.kernel = 1 if kernel == "coo" else 0
        o.value_map = int(bool(value_map))
        o.slices = int(slices)
        o.lds_stage = int(lds_stage)
        o.panels, o.panel_rows, o.panel_waves = int(panels), int(panel_rows), int(panel_waves)
        keep_b = None
        if tile_bounds is not None and len(tile_bounds) > 0:
            keep_b = (ctypes.c_int32 * len(tile_bounds))(*[int(v) for v in tile_bounds])
            o.tile_bounds, o.n_tile_bounds = ctypes.cast(keep_b, vp), len(tile_bounds)
        keep = None
        if wl is None:
            o.wl_policy = 0
        elif isinstance(wl, (int, np.integer)):
            o.wl_policy, o.wl_all = 2, int(wl)
        else:
            keep = (ctypes.c_int32 * len(wl))(*[int(v) for v in wl])
            o.wl_policy, o.wl_per_tile, o.n_wl_per_tile = 1, ctypes.cast(keep, vp), len(wl)
        if perf_table == "default":
            perf_table = DEFAULT_PERF_TABLE if os.path.exists(DEFAULT_PERF_TABLE) else None
        self.perf_table = perf_table
        o.perf_table = perf_table.encode() if perf_table else None
        h = vp()
        c = A.c()
        _check(lib.tc_build_tiled(ctypes.byref(c), ctypes.byref(o), _stream(stream), ctypes.byref(h)),
               "tc_build_tiled")
        self._h = h
        del keep, keep_b

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().tc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("handle is closed")
        return self._h

    # -- queries
    def info(self) -> dict:
        inf = CInfo()
        _check(load_library().tc_handle_info(self.handle, ctypes.byref(inf)), "tc_handle_info")
        return {name: getattr(inf, name) for name, _ in CInfo._fields_}

    def export_format(self, metadata_only: bool = False) -> dict:
        """Host copies of the whole format (keys as the reference builder's).
        metadata_only skips the per-entry and per-row arrays."""
        inf = self.info()
        sizes = dict(inf)
        sizes["n_tiles+1"] = inf["n_tiles"] + 1
        sizes["nnz_coo"] = inf["nnz"] if inf["kernel"] == 1 else 0
        sizes["n_panels+1"] = inf["n_panels"] + 1 if inf["n_panels"] > 0 else 0
        arrays, view = {}, CFormatView()
        for name, dt, sz in _VIEW_FIELDS:
            if metadata_only and sz in ("nnz_pad", "n_rowid", "n_rows_sorted", "n_rows", "n_cols", "nnz_coo"):
                continue
            if sz == "nnz_coo" and inf["kernel"] != 1:
                continue
            a = np.zeros(max(int(sizes[sz]), 0), dt)
            arrays[name] = a
            setattr(view, name, a.ctypes.data_as(vp) if a.size else None)
        _check(load_library().tc_export_format(self.handle, ctypes.byref(view)), "tc_export_format")
        arrays.update(T=inf["n_dense_tiles"], n_tiles_total=inf["n_tiles"], nnz_pad=inf["nnz_pad"],
                      xcd_groups=inf["xcd_groups"], kernel=inf["kernel"],
                      W=inf["tile_width"], S=inf["wave"], split_len=inf["split_len"],
                      relabel=bool(inf["relabel"]), n_rows=inf["n_rows"], n_cols=inf["n_cols"],
                      n_panels=inf["n_panels"], n_col_tiles=inf["n_col_tiles"], panel_rows=inf["panel_rows"],
                      panel_waves=inf["panel_waves"])
        return arrays

    # -- products
    def refresh_values(self, val: torch.Tensor, stream=None) -> None:
        """New values (nnz floats, in the order of the CSR entries the handle
        was built from) for the same pattern; needs value_map=True."""
        v = _need(val, (self.nnz,), "val")
        _check(load_library().tc_refresh_values(self.handle, _ptr(v), _stream(stream)), "tc_refresh_values")
        self._vals = v  # kept alive until the stream has read it

    def spmv(self, x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """y := A x (caller's ids)."""
        _need(x, (self.n_cols,), "x")
        if y is None:
            y = torch.empty(self.n_rows, dtype=torch.float32, device=x.device)
        _need(y, (self.n_rows,), "y")
        _check(load_library().tc_spmv(self.handle, _ptr(x), _ptr(y), _stream(stream)), "tc_spmv")
        return y

    def spmv_internal(self, x: torch.Tensor, y: torch.Tensor, stream=None) -> torch.Tensor:
        _need(x, (self.n_cols,), "x")
        _need(y, (self.n_rows,), "y")
        _check(load_library().tc_spmv_internal(self.handle, _ptr(x), _ptr(y), _stream(stream)), "tc_spmv_internal")
        return y

    def spmv_tiles(self, x: torch.Tensor, y: torch.Tensor, stream=None) -> torch.Tensor:
        """As spmv_internal, one launch per tile (also for row-panel handles)."""
        _need(x, (self.n_cols,), "x")
        _need(y, (self.n_rows,), "y")
        _check(load_library().tc_spmv_tiles(self.handle, _ptr(x), _ptr(y), _stream(stream)), "tc_spmv_tiles")
        return y

    def spmm_internal_noalloc(self, X: torch.Tensor, Y: torch.Tensor, stream=None) -> torch.Tensor:
        """Y := A X in internal ids with no device allocation by the library."""
        if not isinstance(X, torch.Tensor) or X.dim() != 2:
            raise ValueError("X must be a 2-D tensor (n_cols x k)")
        k = int(X.shape[1])
        _need(X, (self.n_cols, k), "X")
        _need(Y, (self.n_rows, k), "Y")
        _check(load_library().tc_spmm_internal_noalloc(self.handle, _ptr(X), _ptr(Y), k, _stream(stream)),
               "tc_spmm_internal_noalloc")
        return Y

    def spmm(self, X: torch.Tensor, Y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Y := A X for X (n_cols x k, row-major)."""
        if not isinstance(X, torch.Tensor) or X.dim() != 2:
            raise ValueError("X must be a 2-D tensor (n_cols x k)")
        k = int(X.shape[1])
        _need(X, (self.n_cols, k), "X")
        if Y is None:
            Y = torch.empty((self.n_rows, k), dtype=torch.float32, device=X.device)
        _need(Y, (self.n_rows, k), "Y")
        _check(load_library().tc_spmm(self.handle, _ptr(X), _ptr(Y), k, _stream(stream)), "tc_spmm")
        return Y

    # -- drivers
    def pagerank(self, c: float = 0.85, tol: float = 0.0, max_iter: int = 50, check_every: int = 1,
                 out: Optional[torch.Tensor] = None, stream=None, raise_not_converged: bool = True):
        p = out if out is not None else torch.empty(self.n_rows, dtype=torch.float32, device="cuda")
        _need(p, (self.n_rows,), "out")
        it, res = i32(0), ctypes.c_double(0.0)
        st = load_library().tc_pagerank(self.handle, c, tol, max_iter, check_every, _ptr(p), ctypes.byref(it),
                                        ctypes.byref(res), _stream(stream))
        if st != TC_ENOTCONV or raise_not_converged:
            _check(st, "tc_pagerank")
        return p, it.value, res.value

    def hits(self, tol: float = 0.0, max_iter: int = 50, check_every: int = 1, stream=None):
        n = self.n_rows // 2
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        h = torch.empty(n, dtype=torch.float32, device="cuda")
        it, res = i32(0), ctypes.c_double(0.0)
        _check(load_library().tc_hits(self.handle, tol, max_iter, check_every, _ptr(a), _ptr(h), ctypes.byref(it),
                                      ctypes.byref(res), _stream(stream)), "tc_hits")
        return a, h, it.value, res.value

    def rwr(self, seeds, c: float = 0.85, tol: float = 0.0, max_iter: int = 30, check_every: int = 1,
            stream=None):
        s = np.ascontiguousarray(seeds, np.int32)
        k = len(s)
        R = torch.empty((self.n_rows, k), dtype=torch.float32, device="cuda")
        it, res = i32(0), ctypes.c_double(0.0)
        _check(load_library().tc_rwr(self.handle, s.ctypes.data_as(vp), k, c, tol, max_iter, check_every, _ptr(R),
                                     ctypes.byref(it), ctypes.byref(res), _stream(stream)), "tc_rwr")
        return R, it.value, res.value

    # -- timing of the tile kernels
    def set_timing(self, enable: bool):
        _check(load_library().tc_set_timing(self.handle, int(enable)), "tc_set_timing")

    def get_timing(self) -> dict:
        t = CTiming()
        _check(load_library().tc_get_timing(self.handle, ctypes.byref(t)), "tc_get_timing")
        return {"tile_kernel_ms": t.tile_kernel_ms, "tile_launches": t.tile_launches, "spmv_calls": t.spmv_calls}


def rwr_multi(mats, seeds, c: float = 0.85, tol: float = 0.0, max_iter: int = 30, check_every: int = 1,
              graph: bool = True, stream=None):
    """RWR on several graphs at once (one query each): returns (list of score
    vectors, iterations, per-graph last L1 change)."""
    n = len(mats)
    hs = (vp * max(n, 1))(*[m.handle for m in mats])
    s = np.ascontiguousarray(seeds, np.int32)
    if s.size != n:
        raise ValueError("one seed per graph")
    outs = [torch.empty(m.n_rows, dtype=torch.float32, device="cuda") for m in mats]
    ptrs = (vp * max(n, 1))(*[o.data_ptr() for o in outs])
    res = (ctypes.c_double * max(n, 1))()
    it = i32(0)
    _check(load_library().tc_rwr_multi(ctypes.cast(hs, vp), n, s.ctypes.data_as(vp), c, tol, max_iter, check_every,
                                       1 if graph else 0, ctypes.cast(ptrs, vp), ctypes.byref(it),
                                       ctypes.cast(res, vp), _stream(stream)),
           "tc_rwr_multi")
    return outs, it.value, np.array(res[:n])


STREAM_SINK_FLOATS = 8192 * 256


def stream_read(buf: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """One streaming read of buf (float32, contiguous, numel a multiple of 4)
    by the library's measurement kernel; sink holds STREAM_SINK_FLOATS floats."""
    if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.dtype == torch.float32 and buf.is_contiguous()):
        raise ValueError("buf must be a contiguous float32 CUDA tensor")
    _need(sink, (STREAM_SINK_FLOATS,), "sink")
    _check(load_library().tc_stream_read(_ptr(buf), buf.numel(), _ptr(sink), _stream(stream)), "tc_stream_read")


def gather_read(x: torch.Tensor, idx: torch.Tensor, val: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """One pass of the library's random-gather measurement kernel: x[idx[e]]
    times val[e] for every entry (idx int32, val float32, same length, a
    multiple of 512); sink holds STREAM_SINK_FLOATS floats."""
    for t, name, dt in ((x, "x", torch.float32), (idx, "idx", torch.int32), (val, "val", torch.float32)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise ValueError("%s must be a contiguous %s CUDA tensor" % (name, dt))
    if idx.numel() != val.numel():
        raise ValueError("idx and val must have the same length")
    _need(sink, (STREAM_SINK_FLOATS,), "sink")
    _check(load_library().tc_gather_read(_ptr(x), x.numel(), _ptr(idx), _ptr(val), idx.numel(), _ptr(sink),
                                         _stream(stream)), "tc_gather_read")


def release_cached_memory() -> int:
    """Return the library's cached device blocks to HIP; bytes released."""
    return int(load_library().tc_release_cached_memory())


def build_tiled(csr, **opts) -> TiledMatrix:
    return TiledMatrix(csr, **opts)
