"""RWR with learned edge weights, differentiable with respect to the weight
parameters (Appendix F, Eq. 9, extended with a hand-written adjoint).

Every entry e = (i, j) of a square pattern A has features f_e (nf of them):

    w_e = softplus(theta . f_e),   W_e = w_e / S_j   (S_j: sum of w over column j),
    r^0 = e_s,   r^{k+1} = c W r^k + (1 - c) e_s,   k < K.

``EdgeWeightedRWR(A, feats, seed, c, K).scores(theta)`` returns r^K as a torch
tensor that autograd can differentiate with respect to theta (a CPU float64
tensor of nf parameters).  The forward keeps only every ``every``-th iterate
(checkpoints); the backward recomputes the iterates in between and runs

    g^k = c W^T g^{k+1}            (tiled SpMV on a build of W^T)
    dL/dW_e += c g^{k+1}_i r^k_j   (per-entry kernel)

then the normalisation and the softplus back to theta.  The per-entry arrays
of the gradient live in A^T's order (the features are gathered into it once),
so the column passes read them contiguously.  Every step runs in the HIP
library (include/tcspmv.h); this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from .tc import CCsr, DeviceCsr, TiledMatrix, _check, _stream, load_library

vp = ctypes.c_void_p


def _ptr(t: Optional[torch.Tensor]):
    return vp(t.data_ptr()) if t is not None else vp(None)


class EdgeWeightedRWR:
    """Pattern, features and the transposed structure, built once.  The first
    forward builds the tiled formats of W and W^T (with value maps); later
    forwards only put the new values into them."""

    def __init__(self, pattern, feats, seed: int, c: float = 0.85, K: int = 30, every: int = 6,
                 build_opts: Optional[dict] = None, stream=None):
        n_rows, n_cols, rp, col = pattern[:4]
        if n_rows != n_cols:
            raise ValueError("RWR needs a square pattern")
        self.n, self.seed, self.c, self.K, self.every = int(n_rows), int(seed), float(c), int(K), int(every)
        dev = torch.device("cuda")
        self.rp = torch.as_tensor(np.asarray(rp, np.int64)).to(dev) if not torch.is_tensor(rp) else rp.to(dev)
        self.col = torch.as_tensor(np.asarray(col, np.int32)).to(dev) if not torch.is_tensor(col) else col.to(dev)
        self.nnz = int(self.col.numel())
        f = torch.as_tensor(np.asarray(feats, np.float32)) if not torch.is_tensor(feats) else feats
        self.feats = f.to(dev, torch.float32).contiguous().view(self.nnz, -1)
        self.nf = int(self.feats.shape[1])
        self.opts = dict(build_opts or {})
        self.stream = stream
        lib = load_library()
        n, nnz = self.n, self.nnz
        self.rpT = torch.empty(n + 1, dtype=torch.int64, device=dev)
        self.colT = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        permT = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        ones = torch.ones(max(nnz, 1), dtype=torch.float32, device=dev)
        A = CCsr(n, n, nnz, self.rp.data_ptr(), self.col.data_ptr(), ones.data_ptr())
        _check(lib.tc_csr_transpose(ctypes.byref(A), _ptr(self.rpT), _ptr(self.colT), vp(None), _ptr(permT),
                                    _stream(stream)), "tc_csr_transpose")
        self.featsT = torch.empty_like(self.feats)
        _check(lib.tc_gather_rows(_ptr(self.feats), nnz, _ptr(permT), nnz, self.nf, _ptr(self.featsT),
                                  _stream(stream)), "tc_gather_rows")
        del permT, ones
        self.z = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)  # A^T's order
        self.w = torch.empty_like(self.z)
        self.S = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        self.val = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)
        self.valT = torch.empty_like(self.val)
        self.W = self.Wt = None
        self.ckpt = None
        # forwards run so far: the checkpoints, weights and formats belong to
        # the latest one, so a backward for an earlier forward recomputes them
        self.generation = 0

    def close(self):
        for m in (self.W, self.Wt):
            if m is not None:
                m.close()
        self.W = self.Wt = None

    # -- the steps, each one library call
    def _weights(self, theta: np.ndarray):
        th = np.ascontiguousarray(theta, np.float64)
        if th.size != self.nf:
            raise ValueError("theta must have one entry per feature")
        _check(load_library().tc_rwr_edge_weights(self.n, self.nnz, _ptr(self.col), _ptr(self.rpT), self.nf,
                                                  _ptr(self.feats), _ptr(self.featsT), th.ctypes.data_as(vp),
                                                  _ptr(self.z), _ptr(self.w), _ptr(self.S), _ptr(self.val),
                                                  _ptr(self.valT), _stream(self.stream)),
               "tc_rwr_edge_weights")
        n = self.n
        refresh = self.opts.get("kernel", "composite") == "composite"
        if refresh and self.W is not None:
            # same pattern, new values: put them into the existing formats
            self.W.refresh_values(self.val[:self.nnz], stream=self.stream)
            self.Wt.refresh_values(self.valT[:self.nnz], stream=self.stream)
            return
        self.close()
        self.W = TiledMatrix(DeviceCsr((n, n, self.rp, self.col, self.val[:self.nnz])), stream=self.stream,
                             value_map=refresh, **self.opts)
        self.Wt = TiledMatrix(DeviceCsr((n, n, self.rpT, self.colT[:self.nnz], self.valT[:self.nnz])),
                              stream=self.stream, value_map=refresh, **self.opts)

    def forward(self, theta: np.ndarray) -> torch.Tensor:
        self.generation += 1
        self._weights(theta)
        m = (self.K + self.every - 1) // self.every
        self.ckpt = torch.empty((max(m, 1), self.n), dtype=torch.float32, device="cuda")
        rK = torch.empty(self.n, dtype=torch.float32, device="cuda")
        _check(load_library().tc_rwr_iterates(self.W.handle, self.seed, self.c, self.K, self.every,
                                              _ptr(self.ckpt), _ptr(rK), _stream(self.stream)), "tc_rwr_iterates")
        return rK

    def backward(self, gK: torch.Tensor) -> np.ndarray:
        """dL/dtheta for dL/dr^K = gK (after a forward with the same theta)."""
        lib = load_library()
        gK = gK.to(device="cuda", dtype=torch.float32).contiguous()
        if gK.numel() != self.n:
            raise ValueError("dL/dr^K must have n entries")
        G = torch.empty(max(self.nnz, 1), dtype=torch.float64, device="cuda")
        _check(lib.tc_rwr_adjoint(self.W.handle, self.Wt.handle, _ptr(self.rpT), _ptr(self.colT), self.seed,
                                  self.c, self.K, self.every, _ptr(self.ckpt), _ptr(gK), _ptr(G), vp(None),
                                  _stream(self.stream)), "tc_rwr_adjoint")
        out = np.zeros(self.nf, np.float64)
        _check(lib.tc_rwr_theta_grad(self.n, self.nnz, _ptr(self.rpT), self.nf, _ptr(self.featsT), _ptr(self.z),
                                     _ptr(self.w), _ptr(self.S), _ptr(G), self.c, out.ctypes.data_as(vp),
                                     _stream(self.stream)), "tc_rwr_theta_grad")
        return out

    def scores(self, theta: torch.Tensor) -> torch.Tensor:
        """r^K for theta, differentiable with respect to theta."""
        return _RWRFunction.apply(theta, self)


class _RWRFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, model):
        ctx.model = model
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        ctx.theta = theta.detach().cpu().double().numpy().copy()
        out = model.forward(ctx.theta)
        ctx.generation = model.generation
        return out

    @staticmethod
    def backward(ctx, grad_rK):
        model = ctx.model
        if model.generation != ctx.generation:
            # another forward ran since this one: its weights and checkpoints
            # replaced ours, so rebuild them for this theta first
            model.forward(ctx.theta)
            ctx.generation = model.generation
        g = model.backward(grad_rK)
        return torch.from_numpy(g).to(dtype=ctx.theta_dtype, device=ctx.theta_device), None
